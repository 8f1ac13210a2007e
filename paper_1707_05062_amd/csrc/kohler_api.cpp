// C-ABI layer of the Köhler contrast-curve library: contexts, argument checks, launch plans, the
// single-image, asynchronous and batched entry points and the autotuner declared in
// include/kohler.h. The serving loop is in kohler_server.cpp.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "kohler.h"
#include "kohler_host.h"
#include "kohler_impl.h"

using namespace kohler;

namespace kohler {

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
    if (pl.form != FORM_BAND && pl.form != FORM_MARG && pl.form != FORM_TRI) return false;
    if (pl.form == FORM_BAND && (M > kMaxMBand || pl.band < 1 || pl.band > kMaxBandRows)) return false;
    if (pl.form == FORM_TRI && M > kMaxMBand) return false;
    if (pl.form == FORM_MARG && M > kMaxMMarg) return false;
    if (pl.block != 256 && pl.block != 512 && pl.block != 1024) return false;
    if (pl.copies != 1 && pl.copies != 2 && pl.copies != 4) return false;
    if (pl.form == FORM_TRI && pl.copies != 1) return false;
    if (pl.form == FORM_MARG && pl.copies > 2) return false;
    if (pl.acc_split != 0 && pl.acc_split != 1) return false;
    if (pl.grid < 0 || pl.grid > 65535) return false;
    if (pl.replicas < 0 || pl.replicas > kMaxReplicas) return false;
    if (dtype == KOHLER_U8 && pl.px_per_lane != 4 && pl.px_per_lane != 8) return false;
    if (dtype == KOHLER_U16 && pl.px_per_lane != 4) return false;
    return true;
}

kohler_plan default_plan(int dtype, int32_t M) {
    kohler_plan pl{};
    pl.form = (M <= kMaxMBand) ? FORM_BAND : FORM_MARG;
    pl.band = std::min(31, std::max(1, M - 1));  // band + 1 a power of two: exact large-gap test
    pl.block = 512;
    pl.grid = 0;
    pl.px_per_lane = 4;
    pl.replicas = 0;
    pl.copies = pl.form == FORM_BAND ? 2 : 1;
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
    if ((pl.form == FORM_BAND || pl.form == FORM_TRI) && M > kMaxMBand) pl = default_plan(dtype, M);
    if (pl.replicas == 0) pl.replicas = -1;  // filled in below, once the grid is known
    if (pl.grid == 0) {
        const int per_cu = blocks_per_cu(dtype, nbhd, pl.form, pl.px_per_lane, M, pl.band, pl.block, pl.copies);
        const int64_t waves = pl.block / 64;
        const int64_t want = (total_units + waves * 4 - 1) / (waves * 4);  // >= 4 rows per wave
        pl.grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * per_cu));
    }
    pl.grid = std::max(pl.grid, min_grid_for(pl, nbhd, total_units));
    if (pl.replicas < 0) pl.replicas = replicas_for(pl.grid);
    return pl;
}

// Every LDS counter of a workgroup is 32 bits: it counts at most w per pixel the workgroup sees
// (pairs per pixel, or the degree weight of the marginal form), and a workgroup sees about
// units / grid tile rows (plus one chunk), so half the counter range bounds the grid from below.
int min_grid_for(const kohler_plan &pl, int32_t nbhd, int64_t units) {
    const int64_t w = pl.form == FORM_MARG ? 8 : (nbhd == 4 ? 2 : 4);
    const int64_t g = (w * 64 * pl.px_per_lane * units + (int64_t(1) << 31) - 1) >> 31;
    return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65535);
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

}  // namespace kohler

namespace {

int launch(kohler_ctx *ctx, const KParams &base, int dtype, int32_t nbhd, const kohler_plan &pl,
           hipStream_t stream) {
    KParams p = base;
    p.band = pl.band;
    p.copies = pl.copies;
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
        case KOHLER_E_CANCELED: return "request cancelled";
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
    (void)hipFree(ctx->level_hist);
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
    if ((pl.form == FORM_MARG || pl.form == FORM_TRI) && pl.band == 0) pl.band = 1;
    if (pl.copies == 0) pl.copies = pl.form == FORM_BAND ? 2 : 1;
    if (!valid_plan(pl, dtype, M)) return KOHLER_E_ARG;
    if (lds_bytes(pl.form, M, pl.band, pl.block, pl.copies) > kMaxLdsBytes) return KOHLER_E_ARG;
    if (pl.block > max_block_for(dtype, nbhd, pl.form, pl.px_per_lane, M)) return KOHLER_E_ARG;
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
    p.packed_acc = (!pl.acc_split && packable(H, W, nbhd)) ? 1 : 0;
    p.nrep = pl.replicas;
    p.rep_stride = replica_stride(M);
    p.acc_stride = (int64_t)p.nrep * p.rep_stride;
    p.total_units = p.img0.nunits;
    p.acc = ctx->acc1;
    p.done = ctx->done1;
    p.rflag = ctx->rflag1;
    p.dyn = 1;
    p.ostride = M;
    p.istride = 1;
    p.thr_stride = thr_capacity;
    p.sum = d_sum;
    p.count = d_count;
    p.C = d_C;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.t0 = d_t0;
    p.status = d_status;
    return launch(ctx, p, dtype, nbhd, pl, stream);
}

// ------------------------------------------------------------------------------------------------
// Other neighbourhoods and the pre-filter

namespace {

// The kernel's offset tables for a neighbourhood description; false if the description is invalid.
bool nbhd_params(const kohler_nbhd &nb, NbParams &q) {
    int hy[2][kNbMaxHalf], hx[2][kNbMaxHalf], nh[2];
    if (nb.kind == KOHLER_NBHD_HEX6) {
        // odd rows shifted right by half a pixel: (0, 1), then the two touching pixels of the row below
        static const int EY[3] = {0, 1, 1}, EX[3] = {1, -1, 0}, OY[3] = {0, 1, 1}, OX[3] = {1, 0, 1};
        for (int a = 0; a < 3; ++a) {
            hy[0][a] = EY[a], hx[0][a] = EX[a];
            hy[1][a] = OY[a], hx[1][a] = OX[a];
        }
        nh[0] = nh[1] = 3;
    } else if (nb.kind == KOHLER_NBHD_OFFSETS) {
        if (nb.n_half < 1 || nb.n_half > KOHLER_NBHD_MAX_HALF) return false;
        for (int a = 0; a < nb.n_half; ++a) {
            int dy = nb.half_dy[a], dx = nb.half_dx[a];
            if (dy == 0 && dx == 0) return false;
            if (dy < -kNbMaxRadius || dy > kNbMaxRadius || dx < -kNbMaxRadius || dx > kNbMaxRadius) return false;
            if (dy < 0 || (dy == 0 && dx < 0)) dy = -dy, dx = -dx;  // the same unordered pairs
            for (int b = 0; b < a; ++b)
                if (hy[0][b] == dy && hx[0][b] == dx) return false;  // an offset given twice (or with its negation)
            hy[0][a] = hy[1][a] = dy;
            hx[0][a] = hx[1][a] = dx;
        }
        nh[0] = nh[1] = nb.n_half;
    } else {
        return false;
    }
    // the whole neighbourhood of a pixel in a row of parity par: its half offsets, and the negated
    // half offsets of the row each one comes from (y - dy)
    q.radius = 0;
    for (int par = 0; par < 2; ++par) {
        q.nhalf[par] = nh[par];
        int nf = 0;
        for (int a = 0; a < nh[par]; ++a) {
            q.hdy[par][a] = (int8_t)hy[par][a];
            q.hdx[par][a] = (int8_t)hx[par][a];
            q.fdy[par][nf] = (int8_t)hy[par][a];
            q.fdx[par][nf++] = (int8_t)hx[par][a];
            q.radius = std::max(q.radius, std::max(hy[par][a], std::abs(hx[par][a])));
        }
        for (int src = 0; src < 2; ++src)
            for (int a = 0; a < nh[src]; ++a)
                if (((hy[src][a] & 1) ? 1 - par : par) == src) {  // row y - dy has parity src
                    q.fdy[par][nf] = (int8_t)-hy[src][a];
                    q.fdx[par][nf++] = (int8_t)-hx[src][a];
                }
        q.nfull[par] = nf;
    }
    return true;
}

}  // namespace

int kohler_curve_nbhd_async(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                            int32_t M, const kohler_nbhd *nbhd, int32_t prefilter, int64_t *d_sum,
                            int64_t *d_count, double *d_C, int32_t *d_thr, int32_t thr_capacity,
                            int32_t *d_n_thr, int32_t *d_t0, int32_t *d_status, kohler_stream_t stream) {
    if (!ctx || !d_img || !nbhd || !valid_shape(dtype, H, W, pitch, M, 4)) return KOHLER_E_ARG;
    if (M > kNbMaxM || (prefilter != 0 && prefilter != 1)) return KOHLER_E_ARG;
    if (!d_sum || !d_count || !d_C || !d_n_thr || !d_t0 || !d_status) return KOHLER_E_ARG;
    if (thr_capacity < 0 || (thr_capacity > 0 && !d_thr)) return KOHLER_E_ARG;
    NbParams q{};
    if (!nbhd_params(*nbhd, q)) return KOHLER_E_ARG;
    const int form = M <= kMaxMBand ? FORM_TRI : FORM_MARG;
    const int block = kNbBlock;
    q.filter = prefilter;
    q.k.M = M;
    const size_t lds = nbhd_lds_layout(q, form, block);
    if (lds > kMaxLdsBytes) return KOHLER_E_ARG;
    q.tiles_x = (W + block - 1) / block;
    q.tiles = ((H + q.tile_rows - 1) / q.tile_rows) * q.tiles_x;
    const int nmax = std::max(q.nhalf[0], q.nhalf[1]);
    // LDS counters are 32-bit: a workgroup sees at most 4 * nmax increments per pixel (a pair's
    // counters, or a pixel's degree in the marginal form)
    const int64_t px_per_wg_max = (int64_t(1) << 31) / (4 * nmax);
    const int64_t min_grid = (H * W + px_per_wg_max - 1) / px_per_wg_max + 1;
    const int per_cu = nbhd_blocks_per_cu(dtype, form, M, block, lds);
    int64_t grid = std::min<int64_t>(q.tiles, (int64_t)ctx->num_cus * per_cu);
    grid = std::max<int64_t>(grid, std::min<int64_t>(min_grid, q.tiles));
    if (grid > 65535) return KOHLER_E_ARG;

    KParams &p = q.k;
    p.imgs = nullptr;
    p.img0 = describe(d_img, dtype, H, W, pitch, 4, 0);
    p.n = 1;
    p.cap = thr_capacity;
    p.packed_acc = (int64_t)nmax * H * W < (int64_t(1) << 30) ? 1 : 0;
    p.nrep = replicas_for((int)grid);
    p.rep_stride = replica_stride(M);
    p.acc_stride = (int64_t)p.nrep * p.rep_stride;
    p.total_units = q.tiles;
    p.acc = ctx->acc1;
    p.done = ctx->done1;
    p.rflag = ctx->rflag1;
    p.dyn = 1;
    p.band = 1;
    p.copies = 1;
    p.ostride = M;
    p.istride = 1;
    p.thr_stride = thr_capacity;
    p.sum = d_sum;
    p.count = d_count;
    p.C = d_C;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.t0 = d_t0;
    p.status = d_status;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    return pick_status(launch_nbhd(q, dtype, form, block, (int)grid, lds, reinterpret_cast<hipStream_t>(stream)));
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
    int nrep = pl.replicas;
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
        ctx->h_table[i].out = i;
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
    p.packed_acc = pl.acc_split ? 0 : 1;
    for (int32_t i = 0; i < n; ++i)
        if (!packable(H[i], W[i], nbhd)) p.packed_acc = 0;
    p.nrep = nrep;
    p.rep_stride = rstride;
    p.acc_stride = (int64_t)nrep * rstride;
    p.total_units = ustart;
    p.ostride = M;
    p.istride = 1;
    p.thr_stride = thr_capacity;
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

// ------------------------------------------------------------------------------------------------
// Autotuner: coordinate descent over the plan knobs, timing each candidate on the caller's workload.

int kohler_autotune(kohler_ctx *ctx, int32_t n, const void *const *d_imgs, const int64_t *H,
                    const int64_t *W, const int64_t *pitch, int dtype, int32_t M, int32_t nbhd,
                    int32_t reps, kohler_plan *best, double *best_us) {
    if (!ctx || n < 1 || !d_imgs || !H || !W || !pitch || !best || reps < 0 || reps > 1000) return KOHLER_E_ARG;
    for (int32_t i = 0; i < n; ++i)
        if (!d_imgs[i] || !valid_shape(dtype, H[i], W[i], pitch[i], M, nbhd)) return KOHLER_E_ARG;
    if (reps == 0) reps = 5;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);

    const auto key = std::make_tuple(dtype, (int)M, (int)nbhd);
    bool had_plan = false;
    kohler_plan saved{};
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->plans.find(key);
        if (it != ctx->plans.end()) {
            had_plan = true;
            saved = it->second;
        }
    }
    auto restore = [&]() {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (had_plan) ctx->plans[key] = saved;
        else ctx->plans.erase(key);
    };

    // trial outputs: image-major arrays as kohler_curve_batch writes them
    const int32_t cap = M / 2 + 1;
    const size_t words = (size_t)n * (3 * (size_t)M + 2 + (size_t)(cap + 1) / 2 + 2);
    int64_t *buf = nullptr;
    if ((e = hipMalloc(&buf, words * sizeof(int64_t))) != hipSuccess) return pick_status(e);
    int64_t *d_sum = buf, *d_count = buf + (size_t)n * M;
    double *d_C = reinterpret_cast<double *>(buf + (size_t)2 * n * M);
    int32_t *d_int = reinterpret_cast<int32_t *>(buf + (size_t)3 * n * M);
    int32_t *d_n = d_int, *d_t0 = d_int + n, *d_st = d_int + 2 * n, *d_thr = d_int + 4 * n;
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);

    auto run_once = [&]() -> int {
        if (n == 1)
            return kohler_curve_async(ctx, d_imgs[0], dtype, H[0], W[0], pitch[0], M, nbhd, d_sum, d_count,
                                      d_C, d_thr, cap, d_n, d_t0, d_st, ctx->stream);
        return kohler_curve_batch(ctx, n, d_imgs, H, W, pitch, dtype, M, nbhd, d_sum, d_count, d_C, d_thr,
                                  cap, d_n, d_t0, d_st, ctx->stream);
    };
    // median launch time of a plan in microseconds, or a negative status
    std::map<std::tuple<int, int, int, int, int, int, int>, double> seen;
    auto time_plan = [&](const kohler_plan &pl, double *us) -> int {
        const auto k = std::make_tuple(pl.form, pl.band, pl.block, pl.grid, pl.px_per_lane, pl.replicas, pl.copies);
        auto it = seen.find(k);
        if (it != seen.end()) {
            *us = it->second;
            return KOHLER_OK;
        }
        int st = kohler_set_plan(ctx, dtype, M, nbhd, &pl);
        if (st != KOHLER_OK) return st;
        for (int w = 0; w < 2 && st == KOHLER_OK; ++w) st = run_once();
        for (int r = 0; r < reps && st == KOHLER_OK; ++r) {
            if ((e = hipEventRecord(ev[2 * r], ctx->stream)) != hipSuccess) return pick_status(e);
            st = run_once();
            if ((e = hipEventRecord(ev[2 * r + 1], ctx->stream)) != hipSuccess) return pick_status(e);
        }
        if (st != KOHLER_OK) return st;
        if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return pick_status(e);
        std::vector<float> ms((size_t)reps);
        for (int r = 0; r < reps; ++r)
            if ((e = hipEventElapsedTime(&ms[r], ev[2 * r], ev[2 * r + 1])) != hipSuccess) return pick_status(e);
        std::sort(ms.begin(), ms.end());
        *us = 1000.0 * ms[(size_t)reps / 2];
        seen[k] = *us;
        return KOHLER_OK;
    };

    // candidate values of each knob
    std::vector<std::pair<int, int>> shapes;  // (form, band)
    if (M <= kMaxMBand)
        for (int b : {7, 15, 23, 31, 47, 63})  // band + 1 = 2^k keeps the row's large-gap test exact
            if (b <= std::max(1, M - 1)) shapes.emplace_back(FORM_BAND, b);
    if (M <= kMaxMBand) shapes.emplace_back(FORM_TRI, 1);
    if (M <= kMaxMMarg) shapes.emplace_back(FORM_MARG, 1);
    std::vector<int> ppls = dtype == KOHLER_U8 ? std::vector<int>{4, 8} : std::vector<int>{4};
    const std::vector<int> blocks = {256, 512, 1024};
    const std::vector<int> reps_knob = {0, 1, 2, 4, 8, 16};

    kohler_plan cur = default_plan(dtype, M);
    double cur_us = 0.0;
    int st = (e == hipSuccess) ? time_plan(cur, &cur_us) : pick_status(e);
    for (int pass = 0; pass < 2 && st == KOHLER_OK; ++pass) {
        auto try_plan = [&](kohler_plan pl) {
            if (st != KOHLER_OK) return;
            double us = 0.0;
            const int r = time_plan(pl, &us);
            if (r == KOHLER_E_ARG) return;  // not a valid plan for this family (e.g. LDS too large)
            if (r != KOHLER_OK) {
                st = r;
                return;
            }
            if (us < cur_us) {
                cur = pl;
                cur_us = us;
            }
        };
        const kohler_plan base_shape = cur;
        for (auto fb : shapes) {
            kohler_plan pl = base_shape;
            pl.form = fb.first;
            pl.band = fb.second;
            if (pl.form != FORM_BAND) pl.copies = 1;
            else if (base_shape.form != FORM_BAND) pl.copies = 2;
            try_plan(pl);
        }
        if (cur.form != FORM_TRI) {  // table copies: 1, 2 or 4 (banded), 1 or 2 (marginal, as LDS allows)
            const kohler_plan base_copies = cur;
            for (int v : {1, 2, 4}) {
                if (cur.form == FORM_MARG && v > 2) continue;
                kohler_plan pl = base_copies;
                pl.copies = v;
                try_plan(pl);
            }
        }
        const kohler_plan base_ppl = cur;
        for (int v : ppls) {
            kohler_plan pl = base_ppl;
            pl.px_per_lane = v;
            try_plan(pl);
        }
        const kohler_plan base_block = cur;
        for (int v : blocks) {
            kohler_plan pl = base_block;
            pl.block = v;
            try_plan(pl);
        }
        // grid: automatic, or 1..4 workgroups per compute unit within the occupancy limit
        const kohler_plan base_grid = cur;
        const int per_cu = blocks_per_cu(dtype, nbhd, cur.form, cur.px_per_lane, M, cur.band, cur.block, cur.copies);
        for (int v = 0; v <= std::min(4, per_cu); ++v) {
            kohler_plan pl = base_grid;
            pl.grid = v * ctx->num_cus;
            try_plan(pl);
        }
        const kohler_plan base_rep = cur;
        for (int v : reps_knob) {
            kohler_plan pl = base_rep;
            pl.replicas = v;
            try_plan(pl);
        }
    }
    // strip width, band, grid and merge schedule interact (occupancy, replicas per workgroup
    // count): a last joint sweep over them for the chosen form and block
    if (st == KOHLER_OK) {
        const kohler_plan base = cur;
        std::vector<int> bands = {base.band};
        if (base.form == FORM_BAND)
            for (int b : {15, 31, 47, 63})
                if (b != base.band && b <= std::max(1, M - 1)) bands.push_back(b);
        for (int bv : bands)
            for (int pv : ppls) {
                const int per_cu = blocks_per_cu(dtype, nbhd, base.form, pv, M, bv, base.block, base.copies);
                for (int gv = 0; gv <= std::min(4, per_cu); ++gv)
                    for (int rv : {1, 2, 4, 8}) {
                        if (st != KOHLER_OK) break;
                        kohler_plan pl = base;
                        pl.band = bv;
                        pl.px_per_lane = pv;
                        pl.grid = gv * ctx->num_cus;
                        pl.replicas = rv;
                        double us = 0.0;
                        const int r = time_plan(pl, &us);
                        if (r == KOHLER_E_ARG) continue;
                        if (r != KOHLER_OK) {
                            st = r;
                            break;
                        }
                        if (us < cur_us) {
                            cur = pl;
                            cur_us = us;
                        }
                    }
            }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    (void)hipFree(buf);
    if (st != KOHLER_OK) {
        restore();
        return st;
    }
    st = kohler_set_plan(ctx, dtype, M, nbhd, &cur);
    if (st != KOHLER_OK) {
        restore();
        return st;
    }
    *best = cur;
    if (best_us) *best_us = cur_us;
    return KOHLER_OK;
}

}  // extern "C"
