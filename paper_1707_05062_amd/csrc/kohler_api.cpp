// C-ABI layer of the Köhler contrast-curve library: contexts, argument checks, launch plans and the
// single-image, asynchronous and batched entry points declared in include/kohler.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "kohler.h"
#include "kohler_impl.h"

using namespace kohler;

struct kohler_ctx {
    int device = 0;
    int num_cus = 256;
    hipStream_t stream = nullptr;

    // single-image scratch (largest M), zero between calls
    int64_t *acc1 = nullptr;
    unsigned long long *done1 = nullptr;
    uint32_t *rflag1 = nullptr;

    // batch scratch, grown to the largest (n, M) seen
    size_t batch_acc_words = 0;
    int32_t batch_n = 0;
    int64_t *accb = nullptr;
    unsigned long long *doneb = nullptr;
    uint32_t *rflagb = nullptr;
    KImage *d_table = nullptr;
    KImage *h_table = nullptr;  // pinned
    int32_t table_cap = 0;

    // synchronous entry point: device copy of a host image, device outputs, pinned host outputs
    void *d_img = nullptr;
    size_t d_img_bytes = 0;
    int64_t *d_out_sc = nullptr;  // sum[M], count[M]
    double *d_out_C = nullptr;
    int32_t *d_out_i = nullptr;   // n_thr, t0, status
    int32_t *d_thr = nullptr;
    int32_t d_thr_cap = 0;
    int64_t *h_out_sc = nullptr;
    double *h_out_C = nullptr;
    int32_t *h_out_i = nullptr;
    int32_t *h_thr = nullptr;
    int32_t h_thr_cap = 0;

    std::map<std::tuple<int, int, int>, kohler_plan> plans;
    std::mutex mu;
};

namespace {

constexpr int kMaxM = std::max(kMaxMBand, kMaxMMarg);

int pick_status(hipError_t e) {
    if (e == hipSuccess) return KOHLER_OK;
    if (e == hipErrorOutOfMemory) return KOHLER_E_NOMEM;
    return KOHLER_E_DEVICE;
}

bool valid_shape(int dtype, int64_t H, int64_t W, int64_t pitch, int32_t M, int32_t nbhd) {
    if (dtype != KOHLER_U8 && dtype != KOHLER_U16) return false;
    if (H < 1 || W < 1 || pitch < W) return false;
    if (W > (int64_t(1) << 30)) return false;  // column indices stay 32-bit in the kernels
    if (H > (int64_t(1) << 40) / W) return false;
    if (nbhd != 4 && nbhd != 8) return false;
    if (M < 1) return false;
    if (dtype == KOHLER_U8 && M > 256) return false;
    if (dtype == KOHLER_U16 && M > KOHLER_MAX_M_U16) return false;
    return true;
}

bool valid_plan(const kohler_plan &pl, int dtype, int32_t M) {
    if (pl.form != FORM_BAND && pl.form != FORM_MARG) return false;
    if (pl.form == FORM_BAND && (M > kMaxMBand || pl.band < 1 || pl.band > kMaxBandRows)) return false;
    if (pl.form == FORM_MARG && M > kMaxMMarg) return false;
    if (pl.block != 256 && pl.block != 512) return false;
    if (pl.grid < 0 || pl.grid > 65535) return false;
    if (dtype == KOHLER_U8 && pl.px_per_lane != 4 && pl.px_per_lane != 8) return false;
    if (dtype == KOHLER_U16 && pl.px_per_lane != 4) return false;
    return true;
}

kohler_plan default_plan(int dtype, int32_t M) {
    kohler_plan pl{};
    pl.form = (M <= kMaxMBand) ? FORM_BAND : FORM_MARG;
    pl.band = std::min(32, std::max(1, M - 1));
    pl.block = 512;
    pl.grid = 0;
    pl.px_per_lane = 4;
    (void)dtype;
    return pl;
}

// Plan for a call: the stored plan of the family, else the default; grid filled in.
kohler_plan resolve_plan(kohler_ctx *ctx, int dtype, int32_t M, int32_t nbhd, int64_t total_units) {
    kohler_plan pl;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->plans.find(std::make_tuple(dtype, (int)M, (int)nbhd));
        pl = (it != ctx->plans.end()) ? it->second : default_plan(dtype, M);
    }
    if (pl.form == FORM_BAND && M > kMaxMBand) pl = default_plan(dtype, M);
    if (pl.grid == 0) {
        const int per_cu = blocks_per_cu(dtype, nbhd, pl.form, pl.px_per_lane, M, pl.band, pl.block);
        const int64_t waves = pl.block / 64;
        const int64_t want = (total_units + waves * 4 - 1) / (waves * 4);  // >= 4 rows per wave
        pl.grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * per_cu));
    }
    return pl;
}

// Accumulator replicas for a launch of `grid` workgroups: about 32 workgroups per replica.
int replicas_for(int grid) { return std::max(1, std::min(kMaxReplicas, grid / 32)); }

// One int64 word per grey level can hold both difference arrays (E * 2^32 + D1) while the image
// has fewer than 2^30 neighbour pairs.
bool packable(int64_t H, int64_t W, int32_t nbhd) {
    const int64_t pairs_bound = (nbhd == 4 ? 2 : 4) * H * W;
    return pairs_bound < (int64_t(1) << 30);
}

int64_t strips_of(int64_t W, int px_per_lane) { return (W + 64 * px_per_lane - 1) / (64 * px_per_lane); }

KImage describe(const void *ptr, int dtype, int64_t H, int64_t W, int64_t pitch, int px_per_lane,
                int64_t ustart) {
    KImage im{};
    im.ptr = ptr;
    im.H = H;
    im.W = W;
    im.pitch = pitch;
    im.ustart = ustart;
    im.nstrips = (int32_t)strips_of(W, px_per_lane);
    im.nunits = (int64_t)im.nstrips * H;
    const size_t esz = dtype == KOHLER_U8 ? 1 : 2;
    const size_t vb = esz * (size_t)px_per_lane;
    im.vec_ok = ((reinterpret_cast<uintptr_t>(ptr) % vb) == 0 && ((size_t)pitch * esz) % vb == 0) ? 1 : 0;
    return im;
}

template <typename T>
int grow_device(T **p, size_t &have, size_t want, bool zero) {
    if (want <= have && *p) return KOHLER_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    have = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), want * sizeof(T));
    if (e != hipSuccess) return pick_status(e);
    if (zero) {
        e = hipMemset(*p, 0, want * sizeof(T));
        if (e != hipSuccess) return pick_status(e);
    }
    have = want;
    return KOHLER_OK;
}

int launch(kohler_ctx *ctx, const KParams &base, int dtype, int32_t nbhd, const kohler_plan &pl,
           hipStream_t stream) {
    KParams p = base;
    p.band = pl.band;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    e = launch_curve(p, dtype, nbhd, pl.form, pl.px_per_lane, pl.block, pl.grid, stream);
    return pick_status(e);
}

}  // namespace

extern "C" {

const char *kohler_strerror(int status) {
    switch (status) {
        case KOHLER_OK: return "ok";
        case KOHLER_E_ARG: return "invalid argument";
        case KOHLER_E_RANGE: return "pixel value out of range (>= M)";
        case KOHLER_E_CAPACITY: return "more local maxima than the threshold capacity";
        case KOHLER_E_NOMEM: return "out of memory";
        case KOHLER_E_DEVICE: return "HIP runtime error";
        case KOHLER_E_BUSY: return "admission refused";
        default: return "unknown status";
    }
}

int kohler_create(kohler_ctx **out, int device) {
    if (!out) return KOHLER_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return KOHLER_E_DEVICE;
    if (device < 0 || device >= ndev) return KOHLER_E_ARG;
    kohler_ctx *ctx = new (std::nothrow) kohler_ctx;
    if (!ctx) return KOHLER_E_NOMEM;
    ctx->device = device;
    int st = KOHLER_OK;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
    const size_t acc1_words = (size_t)kMaxReplicas * (size_t)replica_stride(kMaxM);
    if (e == hipSuccess) e = hipMalloc(&ctx->acc1, sizeof(int64_t) * acc1_words);
    if (e == hipSuccess) e = hipMalloc(&ctx->done1, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&ctx->rflag1, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(ctx->acc1, 0, sizeof(int64_t) * acc1_words);
    if (e == hipSuccess) e = hipMemset(ctx->done1, 0, sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(ctx->rflag1, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&ctx->d_out_sc, sizeof(int64_t) * 2 * kMaxM);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_out_C, sizeof(double) * kMaxM);
    if (e == hipSuccess) e = hipMalloc(&ctx->d_out_i, sizeof(int32_t) * 4);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_out_sc, sizeof(int64_t) * 2 * kMaxM, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_out_C, sizeof(double) * kMaxM, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->h_out_i, sizeof(int32_t) * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
        st = pick_status(e);
        kohler_destroy(ctx);
        return st;
    }
    *out = ctx;
    return KOHLER_OK;
}

void kohler_destroy(kohler_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->acc1);
    (void)hipFree(ctx->done1);
    (void)hipFree(ctx->rflag1);
    (void)hipFree(ctx->accb);
    (void)hipFree(ctx->doneb);
    (void)hipFree(ctx->rflagb);
    (void)hipFree(ctx->d_table);
    (void)hipFree(ctx->d_img);
    (void)hipFree(ctx->d_out_sc);
    (void)hipFree(ctx->d_out_C);
    (void)hipFree(ctx->d_out_i);
    (void)hipFree(ctx->d_thr);
    if (ctx->h_table) (void)hipHostFree(ctx->h_table);
    if (ctx->h_out_sc) (void)hipHostFree(ctx->h_out_sc);
    if (ctx->h_out_C) (void)hipHostFree(ctx->h_out_C);
    if (ctx->h_out_i) (void)hipHostFree(ctx->h_out_i);
    if (ctx->h_thr) (void)hipHostFree(ctx->h_thr);
    if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int kohler_set_plan(kohler_ctx *ctx, int dtype, int32_t M, int32_t nbhd, const kohler_plan *plan) {
    if (!ctx || !plan) return KOHLER_E_ARG;
    if (!valid_shape(dtype, 1, 1, 1, M, nbhd)) return KOHLER_E_ARG;
    kohler_plan pl = *plan;
    if (pl.form == 0) {
        const kohler_plan d = default_plan(dtype, M);
        pl.form = d.form;
        if (pl.band == 0) pl.band = d.band;
    }
    if (pl.form == FORM_MARG && pl.band == 0) pl.band = 1;
    if (!valid_plan(pl, dtype, M)) return KOHLER_E_ARG;
    if (lds_bytes(pl.form, M, pl.band, pl.block) > kMaxLdsBytes) return KOHLER_E_ARG;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->plans[std::make_tuple(dtype, (int)M, (int)nbhd)] = pl;
    return KOHLER_OK;
}

int kohler_get_plan(kohler_ctx *ctx, int dtype, int64_t H, int64_t W, int32_t M, int32_t nbhd,
                    kohler_plan *plan) {
    if (!ctx || !plan || !valid_shape(dtype, H, W, W, M, nbhd)) return KOHLER_E_ARG;
    kohler_plan pl0 = resolve_plan(ctx, dtype, M, nbhd, 1);
    const int64_t units = strips_of(W, pl0.px_per_lane) * H;
    *plan = resolve_plan(ctx, dtype, M, nbhd, units);
    return KOHLER_OK;
}

int kohler_curve_async(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W,
                       int64_t pitch, int32_t M, int32_t nbhd, int64_t *d_sum, int64_t *d_count,
                       double *d_C, int32_t *d_thr, int32_t thr_capacity, int32_t *d_n_thr,
                       int32_t *d_t0, int32_t *d_status, kohler_stream_t stream) {
    if (!ctx || !d_img || !valid_shape(dtype, H, W, pitch, M, nbhd)) return KOHLER_E_ARG;
    if (!d_sum || !d_count || !d_C || !d_n_thr || !d_t0 || !d_status) return KOHLER_E_ARG;
    if (thr_capacity < 0 || (thr_capacity > 0 && !d_thr)) return KOHLER_E_ARG;
    kohler_plan pl = resolve_plan(ctx, dtype, M, nbhd, 1);
    const int64_t units = strips_of(W, pl.px_per_lane) * H;
    pl = resolve_plan(ctx, dtype, M, nbhd, units);

    KParams p{};
    p.imgs = nullptr;
    p.img0 = describe(d_img, dtype, H, W, pitch, pl.px_per_lane, 0);
    p.n = 1;
    p.M = M;
    p.cap = thr_capacity;
    p.packed_acc = packable(H, W, nbhd) ? 1 : 0;
    p.nrep = replicas_for(pl.grid);
    p.rep_stride = replica_stride(M);
    p.total_units = p.img0.nunits;
    p.acc = ctx->acc1;
    p.done = ctx->done1;
    p.rflag = ctx->rflag1;
    p.dyn = 1;
    p.sum = d_sum;
    p.count = d_count;
    p.C = d_C;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.t0 = d_t0;
    p.status = d_status;
    return launch(ctx, p, dtype, nbhd, pl, stream);
}

int kohler_curve(kohler_ctx *ctx, const void *img, int dtype, int64_t H, int64_t W, int64_t pitch,
                 int32_t M, int32_t nbhd, int64_t *sum, int64_t *count, double *C,
                 int32_t *thresholds, int32_t thr_capacity, int32_t *n_thresholds, int32_t *t0) {
    if (!ctx || !img || !valid_shape(dtype, H, W, pitch, M, nbhd)) return KOHLER_E_ARG;
    if (!sum || !count || !C || !n_thresholds || !t0) return KOHLER_E_ARG;
    if (thr_capacity < 0 || (thr_capacity > 0 && !thresholds)) return KOHLER_E_ARG;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);

    // a host image goes through the context's device copy first
    const void *dev_img = img;
    hipPointerAttribute_t attr;
    const bool on_device = hipPointerGetAttributes(&attr, img) == hipSuccess &&
                           attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();
    if (!on_device) {
        const size_t esz = dtype == KOHLER_U8 ? 1 : 2;
        const size_t bytes = ((size_t)(H - 1) * (size_t)pitch + (size_t)W) * esz;
        int st = grow_device(reinterpret_cast<uint8_t **>(&ctx->d_img), ctx->d_img_bytes, bytes, false);
        if (st != KOHLER_OK) return st;
        e = hipMemcpyAsync(ctx->d_img, img, bytes, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) return pick_status(e);
        dev_img = ctx->d_img;
    }
    if (thr_capacity > ctx->d_thr_cap) {
        (void)hipFree(ctx->d_thr);
        ctx->d_thr = nullptr;
        ctx->d_thr_cap = 0;
        if ((e = hipMalloc(&ctx->d_thr, sizeof(int32_t) * thr_capacity)) != hipSuccess) return pick_status(e);
        ctx->d_thr_cap = thr_capacity;
    }
    if (thr_capacity > ctx->h_thr_cap) {
        if (ctx->h_thr) (void)hipHostFree(ctx->h_thr);
        ctx->h_thr = nullptr;
        ctx->h_thr_cap = 0;
        if ((e = hipHostMalloc(&ctx->h_thr, sizeof(int32_t) * thr_capacity, hipHostMallocDefault)) != hipSuccess)
            return pick_status(e);
        ctx->h_thr_cap = thr_capacity;
    }
    int st = kohler_curve_async(ctx, dev_img, dtype, H, W, pitch, M, nbhd, ctx->d_out_sc,
                                ctx->d_out_sc + M, ctx->d_out_C, ctx->d_thr, thr_capacity,
                                ctx->d_out_i, ctx->d_out_i + 1, ctx->d_out_i + 2, ctx->stream);
    if (st != KOHLER_OK) return st;
    e = hipMemcpyAsync(ctx->h_out_sc, ctx->d_out_sc, sizeof(int64_t) * 2 * M, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_out_C, ctx->d_out_C, sizeof(double) * M, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_out_i, ctx->d_out_i, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && thr_capacity > 0)
        e = hipMemcpyAsync(ctx->h_thr, ctx->d_thr, sizeof(int32_t) * thr_capacity, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return pick_status(e);
    std::memcpy(sum, ctx->h_out_sc, sizeof(int64_t) * M);
    std::memcpy(count, ctx->h_out_sc + M, sizeof(int64_t) * M);
    std::memcpy(C, ctx->h_out_C, sizeof(double) * M);
    const int32_t n = ctx->h_out_i[0];
    *n_thresholds = n;
    *t0 = ctx->h_out_i[1];
    if (thr_capacity > 0) std::memcpy(thresholds, ctx->h_thr, sizeof(int32_t) * std::min(n, thr_capacity));
    return ctx->h_out_i[2];
}

int kohler_curve_batch(kohler_ctx *ctx, int32_t n, const void *const *d_imgs, const int64_t *H,
                       const int64_t *W, const int64_t *pitch, int dtype, int32_t M, int32_t nbhd,
                       int64_t *d_sum, int64_t *d_count, double *d_C, int32_t *d_thr,
                       int32_t thr_capacity, int32_t *d_n_thr, int32_t *d_t0, int32_t *d_status,
                       kohler_stream_t stream) {
    if (!ctx || n < 1 || !d_imgs || !H || !W || !pitch) return KOHLER_E_ARG;
    if (!d_sum || !d_count || !d_C || !d_n_thr || !d_t0 || !d_status) return KOHLER_E_ARG;
    if (thr_capacity < 0 || (thr_capacity > 0 && !d_thr)) return KOHLER_E_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (!d_imgs[i] || !valid_shape(dtype, H[i], W[i], pitch[i], M, nbhd)) return KOHLER_E_ARG;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);

    kohler_plan pl = resolve_plan(ctx, dtype, M, nbhd, 1);
    int64_t total_units = 0;
    for (int32_t i = 0; i < n; ++i) total_units += strips_of(W[i], pl.px_per_lane) * H[i];
    pl = resolve_plan(ctx, dtype, M, nbhd, total_units);
    // per-image scratch (replicas limited to keep it under 64 MiB) and the descriptor table
    const int64_t rstride = replica_stride(M);
    int nrep = replicas_for(pl.grid);
    while (nrep > 1 && (size_t)n * nrep * rstride > ((size_t)8 << 20)) nrep /= 2;
    const size_t acc_words = (size_t)n * nrep * (size_t)rstride;
    if (acc_words > ctx->batch_acc_words) {
        int st = grow_device(&ctx->accb, ctx->batch_acc_words, acc_words, true);
        if (st != KOHLER_OK) return st;
    }
    if (n > ctx->batch_n) {
        size_t have = 0;
        (void)hipFree(ctx->doneb);
        ctx->doneb = nullptr;
        int st = grow_device(&ctx->doneb, have, (size_t)n, true);
        if (st != KOHLER_OK) return st;
        have = 0;
        (void)hipFree(ctx->rflagb);
        ctx->rflagb = nullptr;
        st = grow_device(&ctx->rflagb, have, (size_t)n, true);
        if (st != KOHLER_OK) return st;
        ctx->batch_n = n;
    }
    if (n > ctx->table_cap) {
        (void)hipFree(ctx->d_table);
        ctx->d_table = nullptr;
        if (ctx->h_table) (void)hipHostFree(ctx->h_table);
        ctx->h_table = nullptr;
        ctx->table_cap = 0;
        if ((e = hipMalloc(&ctx->d_table, sizeof(KImage) * n)) != hipSuccess) return pick_status(e);
        if ((e = hipHostMalloc(&ctx->h_table, sizeof(KImage) * n, hipHostMallocDefault)) != hipSuccess)
            return pick_status(e);
        ctx->table_cap = n;
    }
    // the pinned table may still be read by a previous batch's copy on this stream
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return pick_status(e);
    int64_t ustart = 0;
    for (int32_t i = 0; i < n; ++i) {
        ctx->h_table[i] = describe(d_imgs[i], dtype, H[i], W[i], pitch[i], pl.px_per_lane, ustart);
        ustart += ctx->h_table[i].nunits;
    }
    e = hipMemcpyAsync(ctx->d_table, ctx->h_table, sizeof(KImage) * n, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return pick_status(e);

    KParams p{};
    p.imgs = ctx->d_table;
    p.img0 = ctx->h_table[0];
    p.n = n;
    p.M = M;
    p.cap = thr_capacity;
    p.packed_acc = 1;
    for (int32_t i = 0; i < n; ++i)
        if (!packable(H[i], W[i], nbhd)) p.packed_acc = 0;
    p.nrep = nrep;
    p.rep_stride = rstride;
    p.total_units = ustart;
    p.acc = ctx->accb;
    p.done = ctx->doneb;
    p.rflag = ctx->rflagb;
    p.sum = d_sum;
    p.count = d_count;
    p.C = d_C;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.t0 = d_t0;
    p.status = d_status;
    return launch(ctx, p, dtype, nbhd, pl, stream);
}

}  // extern "C"
