// Serving loop of the Köhler contrast-curve library: the kohler_server_* entry points declared in
// include/kohler.h. Requests are admitted in arrival order when a device slot and room in the image
// arena (the HBM budget) are free; whatever is admitted together goes to the GPU in one persistent
// launch on an idle lane (stream), and a request admitted alone replays a HIP graph built once per
// image shape and lane. Each slot keeps its accumulators and its result record resident in device
// memory; a completed launch's records are copied to pinned host memory by the launch itself and
// picked up by the scheduler thread, which polls the launch's event.

#include <hip/hip_runtime.h>

#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kohler.h"
#include "kohler_host.h"
#include "kohler_impl.h"
#include "kohler_arena.h"

using namespace kohler;

namespace {

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000 + ts.tv_nsec;
}

enum ReqState { QUEUED, RUNNING, DONE };

struct Request {
    const void *img = nullptr;  // what the device reads from: the caller's image or pinned staging
    bool on_device = false;
    void *staging = nullptr;    // pinned copy of a pageable image (owned)
    size_t staging_bytes = 0;
    int64_t H = 0, W = 0, pitch = 0;
    size_t bytes = 0;
    ReqState state = QUEUED;
    int slot = -1;
    bool has_arena = false;
    size_t arena_off = 0;
    int32_t status = KOHLER_OK, n_thr = 0, t0 = -1, batch = 0, graph = 0;
    int64_t t_submit = 0, t_launch = 0, t_issued = 0, t_done = 0;
    std::vector<int64_t> sum, count;
    std::vector<double> C;
    std::vector<int32_t> thr;
    // video mode: where the labels go, and the arena block they pass through for a host destination
    uint8_t *labels = nullptr;
    int64_t lpitch = 0;
    bool labels_on_device = false;
    bool has_label_block = false;
    size_t label_off = 0;
};

// What a launch needs of one admitted request (copied out of the request table before the
// scheduler releases its lock).
struct Item {
    uint64_t ticket;
    const void *img;
    bool on_device;
    int64_t H, W, pitch;
    size_t bytes;
    int slot;
    size_t arena_off;
    uint8_t *labels;       // destination of the labels (video mode), or null
    int64_t lpitch;
    bool labels_on_device;
    size_t label_off;      // arena block the labels pass through (host destination)
};

struct Launch {
    int lane = 0;
    hipEvent_t ev = nullptr;
    KImage *htable = nullptr;  // pinned descriptor table of a batched launch
    bool graph = false;
    bool built = false;        // a graph was built for this launch
    std::vector<uint64_t> tickets;
};

// A graph is specific to an image shape, whether the image is already on the device, the lane and
// the launch plan; buffers and the slot are updated in the instantiated graph before each replay.
typedef std::tuple<int64_t, int64_t, int64_t, int, int, int, int, int, int, int, int, int, int> GraphKey;

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t h2d = nullptr, kern = nullptr, d2h = nullptr;
    // arguments the instantiated graph holds now; a node is updated only when its own change
    const void *src = nullptr;
    const void *img = nullptr;
    int slot = -1;
};

constexpr size_t kMaxGraphs = 64;

}  // namespace

struct kohler_server {
    kohler_ctx *ctx = nullptr;
    kohler_server_config cfg{};
    int device = 0;
    size_t esz = 1;

    // slot state: accumulators, counters and result records, resident for the server's lifetime
    int64_t rstride = 0, acc_words = 0;
    size_t rec_bytes = 0, off_count = 0, off_C = 0, off_int = 0, off_thr = 0;
    int64_t *acc = nullptr;
    unsigned long long *done = nullptr;
    uint32_t *rflag = nullptr;
    uint8_t *rec_dev = nullptr;
    uint8_t *rec_host = nullptr;  // pinned mirror of the records
    size_t slot_state_bytes = 0;

    uint8_t *arena_base = nullptr;
    Arena arena;

    std::vector<hipStream_t> lanes;
    std::vector<int> lane_busy;
    std::vector<KImage *> table_dev;  // per lane: device descriptor table of max_batch entries
    std::vector<KImage *> table_pool; // pinned host tables of max_batch entries
    std::vector<hipEvent_t> ev_pool;
    std::map<GraphKey, GraphEntry> graphs;  // touched by the scheduler thread only

    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    std::vector<int> free_slots;
    std::vector<Launch> inflight;
    std::multimap<size_t, void *> staging_pool;  // free pinned staging buffers by size
    uint64_t next_ticket = 1;
    bool stop = false, paused = false;
    int64_t inflight_reqs = 0;
    kohler_server_counters st{};

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread thread;
};

namespace {

// Kernel arguments for a launch over `items` (all admitted to slots) with plan `pl`.
KParams slot_params(const kohler_server *s, const kohler_plan &pl) {
    KParams p{};
    p.M = s->cfg.M;
    p.band = pl.band;
    p.copies = pl.copies;
    p.cap = s->cfg.thr_capacity;
    p.nrep = pl.replicas;
    p.rep_stride = s->rstride;
    p.acc_stride = s->acc_words;
    p.acc = s->acc;
    p.done = s->done;
    p.rflag = s->rflag;
    p.ostride = (int64_t)(s->rec_bytes / sizeof(int64_t));
    p.istride = (int64_t)(s->rec_bytes / sizeof(int32_t));
    p.thr_stride = p.istride;
    p.sum = reinterpret_cast<int64_t *>(s->rec_dev);
    p.count = reinterpret_cast<int64_t *>(s->rec_dev + s->off_count);
    p.C = reinterpret_cast<double *>(s->rec_dev + s->off_C);
    p.n_thr = reinterpret_cast<int32_t *>(s->rec_dev + s->off_int);
    p.t0 = p.n_thr + 1;
    p.status = p.n_thr + 2;
    p.thr = reinterpret_cast<int32_t *>(s->rec_dev + s->off_thr);
    return p;
}

const void *device_image(const kohler_server *s, const Item &it) {
    return it.on_device ? it.img : static_cast<const void *>(s->arena_base + it.arena_off);
}

// The graph of a one-image launch depends on the image's shape and residence, the lane and the plan.
GraphKey graph_key(const Item &it, int lane, const kohler_plan &pl) {
    return GraphKey(it.H, it.W, it.pitch, it.on_device ? 1 : 0, lane, pl.form, pl.band, pl.block, pl.grid,
                    pl.px_per_lane, pl.replicas, pl.copies, pl.acc_split);
}

// Video mode: after the curve launch on the same stream, the labels of every item that asked for
// them (t0 read from the slot's device record), written to the destination or to the item's arena
// block and copied from there.
hipError_t issue_labels(kohler_server *s, const std::vector<Item> &items, hipStream_t stream) {
    LabelJobs js{};
    js.dtype = s->cfg.dtype;
    auto flush = [&]() -> hipError_t {
        if (js.n == 0) return hipSuccess;
        hipError_t e = launch_label_t0(js, stream);
        js.n = 0;
        return e;
    };
    for (const Item &it : items) {
        if (!it.labels) continue;
        LabelJob &j = js.job[js.n++];
        j.img = device_image(s, it);
        j.labels = it.labels_on_device ? it.labels : s->arena_base + it.label_off;
        j.t0 = reinterpret_cast<const int32_t *>(s->rec_dev + (size_t)it.slot * s->rec_bytes + s->off_int) + 1;
        j.H = it.H;
        j.W = it.W;
        j.pitch = it.pitch;
        j.lpitch = it.labels_on_device ? it.lpitch : it.W;
        if (js.n == kMaxLabelJobs) {
            hipError_t e = flush();
            if (e != hipSuccess) return e;
        }
    }
    hipError_t e = flush();
    for (const Item &it : items) {
        if (e != hipSuccess) break;
        if (it.labels && !it.labels_on_device)
            e = hipMemcpy2DAsync(it.labels, (size_t)it.lpitch, s->arena_base + it.label_off, (size_t)it.W,
                                 (size_t)it.W, (size_t)it.H, hipMemcpyDeviceToHost, stream);
    }
    return e;
}

// Issue one launch (copies in, kernel, copies out, event) on `lane`. Runs without the lock.
int issue(kohler_server *s, int lane, const std::vector<Item> &items, Launch &L) {
    const kohler_server_config &c = s->cfg;
    hipStream_t stream = s->lanes[lane];
    const int n = (int)items.size();
    kohler_plan pl = resolve_plan(s->ctx, c.dtype, c.M, c.nbhd, 1);
    int64_t units = 0;
    bool packed = true;
    for (const Item &it : items) {
        units += strips_of(it.W, pl.px_per_lane) * it.H;
        packed = packed && packable(it.H, it.W, c.nbhd);
    }
    pl = resolve_plan(s->ctx, c.dtype, c.M, c.nbhd, units);
    KParams p = slot_params(s, pl);
    p.packed_acc = (packed && !pl.acc_split) ? 1 : 0;
    p.total_units = units;
    hipError_t e = hipSuccess;

    const bool labelled = std::any_of(items.begin(), items.end(), [](const Item &it) { return it.labels != nullptr; });
    if (n == 1 && c.use_graphs && !labelled && (s->graphs.size() < kMaxGraphs ||
                                   s->graphs.count(graph_key(items[0], lane, pl)))) {
        const Item &it = items[0];
        p.n = 1;
        p.dyn = 1;
        p.img0 = describe(device_image(s, it), c.dtype, it.H, it.W, it.pitch, pl.px_per_lane, 0);
        p.img0.out = it.slot;
        const void *func = nullptr;
        size_t lds = 0;
        if ((e = curve_kernel_for(c.dtype, c.nbhd, pl.form, pl.px_per_lane, c.M, pl.band, pl.block, pl.copies,
                                  &func, &lds)) != hipSuccess)
            return pick_status(e);
        KParams arg = p;
        void *argv[1] = {&arg};
        hipKernelNodeParams kn{};
        kn.func = const_cast<void *>(func);
        kn.gridDim = dim3(pl.grid);
        kn.blockDim = dim3(pl.block);
        kn.sharedMemBytes = (unsigned)lds;
        kn.kernelParams = argv;
        kn.extra = nullptr;
        uint8_t *rec_d = s->rec_dev + (size_t)it.slot * s->rec_bytes;
        uint8_t *rec_h = s->rec_host + (size_t)it.slot * s->rec_bytes;
        void *img_dst = s->arena_base + it.arena_off;

        const GraphKey key = graph_key(it, lane, pl);
        auto found = s->graphs.find(key);
        if (found == s->graphs.end()) {
            GraphEntry g;
            e = hipGraphCreate(&g.graph, 0);
            if (e == hipSuccess && !it.on_device)
                e = hipGraphAddMemcpyNode1D(&g.h2d, g.graph, nullptr, 0, img_dst, it.img, it.bytes,
                                            hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipGraphAddKernelNode(&g.kern, g.graph, g.h2d ? &g.h2d : nullptr, g.h2d ? 1 : 0, &kn);
            if (e == hipSuccess)
                e = hipGraphAddMemcpyNode1D(&g.d2h, g.graph, &g.kern, 1, rec_h, rec_d, s->rec_bytes,
                                            hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (g.exec) (void)hipGraphExecDestroy(g.exec);
                if (g.graph) (void)hipGraphDestroy(g.graph);
                return pick_status(e);
            }
            g.src = it.img;
            g.img = p.img0.ptr;
            g.slot = it.slot;
            found = s->graphs.emplace(key, g).first;
            L.built = true;
        } else {
            // the image's host address changes with every frame; its arena block and the slot
            // usually repeat (first fit, last-freed slot first), and then so do the kernel's
            // arguments and the result copy
            GraphEntry &g = found->second;
            if (!it.on_device && g.src != it.img) {
                e = hipGraphExecMemcpyNodeSetParams1D(g.exec, g.h2d, img_dst, it.img, it.bytes,
                                                      hipMemcpyHostToDevice);
                g.src = it.img;
            }
            if (e == hipSuccess && (g.img != p.img0.ptr || g.slot != it.slot)) {
                e = hipGraphExecKernelNodeSetParams(g.exec, g.kern, &kn);
                g.img = p.img0.ptr;
                // the host-to-device copy's destination moved with the image
                if (e == hipSuccess && !it.on_device)
                    e = hipGraphExecMemcpyNodeSetParams1D(g.exec, g.h2d, img_dst, it.img, it.bytes,
                                                          hipMemcpyHostToDevice);
            }
            if (e == hipSuccess && g.slot != it.slot) {
                e = hipGraphExecMemcpyNodeSetParams1D(g.exec, g.d2h, rec_h, rec_d, s->rec_bytes,
                                                      hipMemcpyDeviceToHost);
                g.slot = it.slot;
            }
            if (e != hipSuccess) {
                g.src = g.img = nullptr;  // unknown state: update every node next time
                g.slot = -1;
                return pick_status(e);
            }
        }
        if ((e = hipGraphLaunch(found->second.exec, stream)) != hipSuccess) return pick_status(e);
        L.graph = true;
    } else {
        for (const Item &it : items)
            if (!it.on_device &&
                (e = hipMemcpyAsync(s->arena_base + it.arena_off, it.img, it.bytes, hipMemcpyHostToDevice,
                                    stream)) != hipSuccess)
                return pick_status(e);
        if (n == 1) {
            const Item &it = items[0];
            p.n = 1;
            p.dyn = 1;
            p.img0 = describe(device_image(s, it), c.dtype, it.H, it.W, it.pitch, pl.px_per_lane, 0);
            p.img0.out = it.slot;
        } else {
            int64_t ustart = 0;
            for (int i = 0; i < n; ++i) {
                const Item &it = items[i];
                L.htable[i] = describe(device_image(s, it), c.dtype, it.H, it.W, it.pitch, pl.px_per_lane, ustart);
                L.htable[i].out = it.slot;
                ustart += L.htable[i].nunits;
            }
            if ((e = hipMemcpyAsync(s->table_dev[lane], L.htable, sizeof(KImage) * n, hipMemcpyHostToDevice,
                                    stream)) != hipSuccess)
                return pick_status(e);
            p.n = n;
            p.dyn = 0;
            p.imgs = s->table_dev[lane];
            p.img0 = L.htable[0];
        }
        if ((e = launch_curve(p, c.dtype, c.nbhd, pl.form, pl.px_per_lane, pl.block, pl.grid, stream)) !=
            hipSuccess)
            return pick_status(e);
        if (labelled && (e = issue_labels(s, items, stream)) != hipSuccess) return pick_status(e);
        for (const Item &it : items)
            if ((e = hipMemcpyAsync(s->rec_host + (size_t)it.slot * s->rec_bytes,
                                    s->rec_dev + (size_t)it.slot * s->rec_bytes, s->rec_bytes,
                                    hipMemcpyDeviceToHost, stream)) != hipSuccess)
                return pick_status(e);
    }
    if ((e = hipEventRecord(L.ev, stream)) != hipSuccess) return pick_status(e);
    return KOHLER_OK;
}

// Release what an admitted request holds (slot, arena block, staging) and mark it done. Lock held.
void retire(kohler_server *s, Request &r, int status) {
    if (r.slot >= 0) {
        if (status == KOHLER_OK) {
            const uint8_t *rec = s->rec_host + (size_t)r.slot * s->rec_bytes;
            const int M = s->cfg.M;
            const int32_t *ints = reinterpret_cast<const int32_t *>(rec + s->off_int);
            r.sum.assign(reinterpret_cast<const int64_t *>(rec), reinterpret_cast<const int64_t *>(rec) + M);
            r.count.assign(reinterpret_cast<const int64_t *>(rec + s->off_count),
                           reinterpret_cast<const int64_t *>(rec + s->off_count) + M);
            r.C.assign(reinterpret_cast<const double *>(rec + s->off_C),
                       reinterpret_cast<const double *>(rec + s->off_C) + M);
            r.n_thr = ints[0];
            r.t0 = ints[1];
            status = ints[2];
            const int32_t keep = std::max(0, std::min(r.n_thr, s->cfg.thr_capacity));
            const int32_t *thr = reinterpret_cast<const int32_t *>(rec + s->off_thr);
            r.thr.assign(thr, thr + keep);
        }
        s->free_slots.push_back(r.slot);
        r.slot = -1;
    }
    if (r.has_arena) {
        s->arena.release(r.arena_off, r.bytes);
        r.has_arena = false;
    }
    if (r.has_label_block) {
        s->arena.release(r.label_off, (size_t)(r.H * r.W));
        r.has_label_block = false;
    }
    if (r.staging) {
        s->staging_pool.emplace(r.staging_bytes, r.staging);
        r.staging = nullptr;
    }
    r.status = status;
    r.state = DONE;
    r.t_done = now_ns();
}

// Completions: every launch whose event has fired. Lock held.
bool reap(kohler_server *s) {
    bool any = false;
    for (size_t k = 0; k < s->inflight.size();) {
        Launch &L = s->inflight[k];
        const hipError_t q = hipEventQuery(L.ev);
        if (q == hipErrorNotReady) {
            ++k;
            continue;
        }
        const int dev_status = (q == hipSuccess) ? KOHLER_OK : KOHLER_E_DEVICE;
        for (uint64_t t : L.tickets) {
            auto it = s->reqs.find(t);
            if (it == s->reqs.end()) continue;
            retire(s, it->second, dev_status);
        }
        s->inflight_reqs -= (int64_t)L.tickets.size();
        s->st.completed += (int64_t)L.tickets.size();
        s->lane_busy[L.lane] = 0;
        s->ev_pool.push_back(L.ev);
        if (L.htable) s->table_pool.push_back(L.htable);
        s->inflight[k] = std::move(s->inflight.back());
        s->inflight.pop_back();
        any = true;
    }
    if (any) s->cv_done.notify_all();
    return any;
}

// Admission: fill idle lanes from the head of the queue. Lock held on entry and exit; released
// while the launch is issued.
bool admit(kohler_server *s, std::unique_lock<std::mutex> &lk) {
    bool any = false;
    const int nl = (int)s->lanes.size();
    for (int lane = 0; lane < nl; ++lane) {
        if (s->lane_busy[lane] || s->stop || s->paused) continue;
        if (s->queue.empty() || s->ev_pool.empty() || s->table_pool.empty()) break;
        std::vector<uint64_t> admitted;
        admit_in_order(s->queue, [&](uint64_t t) -> Request & { return s->reqs.at(t); }, s->arena, s->free_slots,
                       s->cfg.max_batch, admitted);
        std::vector<Item> items;
        const int64_t t_launch = now_ns();
        for (uint64_t t : admitted) {
            Request &r = s->reqs.at(t);
            r.state = RUNNING;
            r.t_launch = t_launch;
            items.push_back(Item{t, r.img, r.on_device, r.H, r.W, r.pitch, r.bytes, r.slot, r.arena_off, r.labels,
                                 r.lpitch, r.labels_on_device, r.label_off});
        }
        if (items.empty()) break;  // no slot or no arena room for the head request
        Launch L;
        L.lane = lane;
        L.ev = s->ev_pool.back();
        s->ev_pool.pop_back();
        L.htable = s->table_pool.back();
        s->table_pool.pop_back();
        s->lane_busy[lane] = 1;
        s->inflight_reqs += (int64_t)items.size();
        s->st.peak_inflight = std::max(s->st.peak_inflight, s->inflight_reqs);

        lk.unlock();
        const int rc = issue(s, lane, items, L);
        lk.lock();

        const int n = (int)items.size();
        const int64_t t_issued = now_ns();
        for (const Item &it : items) {
            Request &r = s->reqs.at(it.ticket);
            r.t_issued = t_issued;
            r.batch = n;
            r.graph = L.graph ? 1 : 0;
            L.tickets.push_back(it.ticket);
        }
        s->st.launches++;
        if (L.graph) s->st.graph_launches++;
        if (L.built) s->st.graphs_built++;
        if (n > 1) s->st.batched_launches++;
        s->st.max_batch_seen = std::max<int64_t>(s->st.max_batch_seen, n);
        if (rc != KOHLER_OK) {
            // nothing of this launch can be trusted: wait for what was queued, then fail it
            (void)hipStreamSynchronize(s->lanes[lane]);
            for (uint64_t t : L.tickets) retire(s, s->reqs.at(t), rc);
            s->inflight_reqs -= n;
            s->st.completed += n;
            s->lane_busy[lane] = 0;
            s->ev_pool.push_back(L.ev);
            s->table_pool.push_back(L.htable);
            s->cv_done.notify_all();
        } else {
            s->inflight.push_back(std::move(L));
        }
        any = true;
    }
    return any;
}

void scheduler(kohler_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool progress = reap(s);
        if (s->stop && s->inflight.empty()) break;
        progress = admit(s, lk) || progress;
        if (progress) continue;
        if (s->inflight.empty()) {
            s->cv_sched.wait(lk);
        } else {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
    // requests still queued at shutdown are cancelled
    while (!s->queue.empty()) {
        Request &r = s->reqs.at(s->queue.front());
        s->queue.pop_front();
        retire(s, r, KOHLER_E_CANCELED);
        s->st.cancelled++;
    }
    s->cv_done.notify_all();
}

void free_all(kohler_server *s) {
    (void)hipSetDevice(s->device);
    for (hipStream_t x : s->lanes)
        if (x) (void)hipStreamSynchronize(x);
    for (auto &kv : s->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (hipEvent_t x : s->ev_pool) (void)hipEventDestroy(x);
    for (KImage *x : s->table_dev) (void)hipFree(x);
    for (KImage *x : s->table_pool) (void)hipHostFree(x);
    for (auto &kv : s->staging_pool) (void)hipHostFree(kv.second);
    for (auto &kv : s->reqs)
        if (kv.second.staging) (void)hipHostFree(kv.second.staging);
    for (hipStream_t x : s->lanes)
        if (x) (void)hipStreamDestroy(x);
    (void)hipFree(s->acc);
    (void)hipFree(s->done);
    (void)hipFree(s->rflag);
    (void)hipFree(s->rec_dev);
    (void)hipFree(s->arena_base);
    if (s->rec_host) (void)hipHostFree(s->rec_host);
    delete s;
}

}  // namespace

extern "C" {

int kohler_server_create(kohler_ctx *ctx, const kohler_server_config *cfg, kohler_server **out) {
    if (!out) return KOHLER_E_ARG;
    *out = nullptr;
    if (!ctx || !cfg) return KOHLER_E_ARG;
    const kohler_server_config c = *cfg;
    if (!valid_shape(c.dtype, 1, 1, 1, c.M, c.nbhd)) return KOHLER_E_ARG;
    if (c.slots < 1 || c.slots > 1024 || c.lanes < 1 || c.lanes > 8) return KOHLER_E_ARG;
    if (c.max_batch < 1 || c.max_batch > c.slots || c.queue_capacity < 1) return KOHLER_E_ARG;
    if (c.thr_capacity < 0 || c.thr_capacity > c.M || c.hbm_budget_bytes <= 0) return KOHLER_E_ARG;

    kohler_server *s = new (std::nothrow) kohler_server;
    if (!s) return KOHLER_E_NOMEM;
    s->ctx = ctx;
    s->cfg = c;
    s->device = ctx->device;
    s->esz = c.dtype == KOHLER_U8 ? 1 : 2;
    s->rstride = replica_stride(c.M);
    s->acc_words = (int64_t)kMaxReplicas * s->rstride;
    // result record of one slot: sum[M] | count[M] | C[M] | n_thr, t0, status, pad | thr[cap]
    s->off_count = (size_t)8 * c.M;
    s->off_C = (size_t)16 * c.M;
    s->off_int = (size_t)24 * c.M;
    s->off_thr = s->off_int + 16;
    s->rec_bytes = round_up(s->off_thr + (size_t)4 * c.thr_capacity, kAlign);
    const size_t S = (size_t)c.slots;
    const size_t acc_bytes = S * (size_t)s->acc_words * sizeof(int64_t);
    const size_t table_bytes = round_up(sizeof(KImage) * (size_t)c.max_batch, kAlign);
    s->slot_state_bytes = acc_bytes + round_up(S * 8, kAlign) + round_up(S * 4, kAlign) + S * s->rec_bytes +
                          (size_t)c.lanes * table_bytes;
    if ((size_t)c.hbm_budget_bytes <= s->slot_state_bytes) {
        delete s;
        return KOHLER_E_ARG;
    }
    const size_t arena_cap = ((size_t)c.hbm_budget_bytes - s->slot_state_bytes) / kAlign * kAlign;

    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipMalloc(&s->acc, acc_bytes);
    if (e == hipSuccess) e = hipMemset(s->acc, 0, acc_bytes);
    if (e == hipSuccess) e = hipMalloc(&s->done, S * 8);
    if (e == hipSuccess) e = hipMemset(s->done, 0, S * 8);
    if (e == hipSuccess) e = hipMalloc(&s->rflag, S * 4);
    if (e == hipSuccess) e = hipMemset(s->rflag, 0, S * 4);
    if (e == hipSuccess) e = hipMalloc(&s->rec_dev, S * s->rec_bytes);
    if (e == hipSuccess) e = hipHostMalloc(&s->rec_host, S * s->rec_bytes, hipHostMallocDefault);
    if (e == hipSuccess && arena_cap) e = hipMalloc(&s->arena_base, arena_cap);
    for (int l = 0; l < c.lanes && e == hipSuccess; ++l) {
        hipStream_t x = nullptr;
        KImage *td = nullptr, *th = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (e == hipSuccess) s->lanes.push_back(x);
        if (e == hipSuccess) e = hipMalloc(&td, table_bytes);
        if (e == hipSuccess) s->table_dev.push_back(td);
        if (e == hipSuccess) e = hipHostMalloc(&th, table_bytes, hipHostMallocDefault);
        if (e == hipSuccess) s->table_pool.push_back(th);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) s->ev_pool.push_back(ev);
    }
    if (e != hipSuccess) {
        const int st = pick_status(e);
        free_all(s);
        return st;
    }
    s->lane_busy.assign((size_t)c.lanes, 0);
    s->arena.reset(arena_cap);
    for (int k = c.slots - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->st.slot_state_bytes = (int64_t)s->slot_state_bytes;
    try {
        s->thread = std::thread(scheduler, s);
    } catch (...) {
        free_all(s);
        return KOHLER_E_NOMEM;
    }
    *out = s;
    return KOHLER_OK;
}

void kohler_server_destroy(kohler_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_sched.notify_all();
    if (s->thread.joinable()) s->thread.join();
    free_all(s);
}

// Both submit entry points: queue one request, with a label destination (video mode) or without.
static int submit_request(kohler_server *s, const void *img, int64_t H, int64_t W, int64_t pitch, uint8_t *labels,
                          int64_t lpitch, uint64_t *ticket) {
    if (!s || !img || !ticket) return KOHLER_E_ARG;
    const kohler_server_config &c = s->cfg;
    if (!valid_shape(c.dtype, H, W, pitch, c.M, c.nbhd)) return KOHLER_E_ARG;
    const size_t bytes = ((size_t)(H - 1) * (size_t)pitch + (size_t)W) * s->esz;
    bool labels_on_device = false;
    if (labels) {
        if (!c.label_t0 || lpitch < W) return KOHLER_E_ARG;
        hipPointerAttribute_t la;
        labels_on_device = hipPointerGetAttributes(&la, labels) == hipSuccess && la.type == hipMemoryTypeDevice;
        (void)hipGetLastError();
        if (!labels_on_device && round_up((size_t)(H * W), kAlign) > s->arena.capacity()) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->st.refused++;
            return KOHLER_E_BUSY;
        }
    }

    hipPointerAttribute_t attr;
    bool on_device = false, pinned = false;
    if (hipPointerGetAttributes(&attr, img) == hipSuccess) {
        on_device = attr.type == hipMemoryTypeDevice;
        pinned = attr.type == hipMemoryTypeHost;
    }
    (void)hipGetLastError();
    const size_t arena_need = (on_device ? 0 : round_up(bytes, kAlign)) +
                              (labels && !labels_on_device ? round_up((size_t)(H * W), kAlign) : 0);
    if (arena_need > s->arena.capacity()) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.refused++;
        return KOHLER_E_BUSY;
    }
    void *staging = nullptr;
    size_t staging_bytes = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= c.queue_capacity) {
            s->st.refused++;
            return KOHLER_E_BUSY;
        }
        if (!on_device && !pinned) {
            auto it = s->staging_pool.lower_bound(bytes);
            if (it != s->staging_pool.end()) {
                staging = it->second;
                staging_bytes = it->first;
                s->staging_pool.erase(it);
            }
        }
    }
    if (!on_device && !pinned) {
        if (!staging) {
            if (hipHostMalloc(&staging, bytes, hipHostMallocDefault) != hipSuccess) return KOHLER_E_NOMEM;
            staging_bytes = bytes;
        }
        std::memcpy(staging, img, bytes);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= c.queue_capacity) {
            if (staging) s->staging_pool.emplace(staging_bytes, staging);
            s->st.refused++;
            return KOHLER_E_BUSY;
        }
        const uint64_t t = s->next_ticket++;
        Request &r = s->reqs[t];
        r.img = staging ? staging : img;
        r.on_device = on_device;
        r.staging = staging;
        r.staging_bytes = staging_bytes;
        r.H = H;
        r.W = W;
        r.pitch = pitch;
        r.bytes = bytes;
        r.labels = labels;
        r.lpitch = lpitch;
        r.labels_on_device = labels_on_device;
        r.t_submit = now_ns();
        s->queue.push_back(t);
        s->st.submitted++;
        *ticket = t;
    }
    s->cv_sched.notify_one();
    return KOHLER_OK;
}

int kohler_server_submit(kohler_server *s, const void *img, int64_t H, int64_t W, int64_t pitch,
                         uint64_t *ticket) {
    return submit_request(s, img, H, W, pitch, nullptr, 0, ticket);
}

int kohler_server_submit_labels(kohler_server *s, const void *img, int64_t H, int64_t W, int64_t pitch,
                                uint8_t *labels, int64_t label_pitch, uint64_t *ticket) {
    if (!labels) return KOHLER_E_ARG;
    return submit_request(s, img, H, W, pitch, labels, label_pitch, ticket);
}

int kohler_server_poll(kohler_server *s, uint64_t ticket) {
    if (!s) return KOHLER_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return KOHLER_E_ARG;
    return it->second.state == DONE ? 1 : 0;
}

int kohler_server_wait(kohler_server *s, uint64_t ticket, int64_t *sum, int64_t *count, double *C,
                       int32_t *thresholds, int32_t thr_capacity, kohler_request_info *info) {
    if (!s || thr_capacity < 0 || (thr_capacity > 0 && !thresholds)) return KOHLER_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return KOHLER_E_ARG;
    Request &r = it->second;  // references into the map stay valid while the element exists
    s->cv_done.wait(lk, [&] { return r.state == DONE; });
    if (!r.sum.empty()) {
        const size_t M = (size_t)s->cfg.M;
        if (sum) std::memcpy(sum, r.sum.data(), M * sizeof(int64_t));
        if (count) std::memcpy(count, r.count.data(), M * sizeof(int64_t));
        if (C) std::memcpy(C, r.C.data(), M * sizeof(double));
        if (thresholds) {
            const size_t k = std::min(r.thr.size(), (size_t)thr_capacity);
            std::memcpy(thresholds, r.thr.data(), k * sizeof(int32_t));
        }
    }
    if (info) {
        info->status = r.status;
        info->n_thresholds = r.n_thr;
        info->t0 = r.t0;
        info->batch = r.batch;
        info->graph = r.graph;
        info->pad = 0;
        info->t_submit_ns = r.t_submit;
        info->t_launch_ns = r.t_launch;
        info->t_issued_ns = r.t_issued;
        info->t_done_ns = r.t_done;
    }
    const int status = r.status;
    s->reqs.erase(it);
    return status;
}

int kohler_server_cancel(kohler_server *s, uint64_t ticket) {
    if (!s) return KOHLER_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return KOHLER_E_ARG;
    Request &r = it->second;
    if (r.state != QUEUED) return KOHLER_E_BUSY;
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), ticket));
    retire(s, r, KOHLER_E_CANCELED);
    s->st.cancelled++;
    s->cv_done.notify_all();
    return KOHLER_OK;
}

int kohler_server_pause(kohler_server *s, int32_t paused) {
    if (!s) return KOHLER_E_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = paused != 0;
    }
    s->cv_sched.notify_all();
    return KOHLER_OK;
}

int kohler_server_stats(kohler_server *s, kohler_server_counters *out) {
    if (!s || !out) return KOHLER_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->arena_bytes = (int64_t)s->arena.capacity();
    out->arena_peak_bytes = (int64_t)s->arena.peak();
    return KOHLER_OK;
}

}  // extern "C"
