// kohler_curve_noalloc: the stream-ordered curve of one image for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc). It is kohler_curve_async without a context: the kernel's scratch (the accumulator
// replicas, the ticket and the range flag) lives in the file-scope device array `scratch` below,
// one copy per GPU, held until the process ends.
//
// Host code never passes `scratch` itself to a kernel (in host code the name is only a stand-in for
// the device symbol): the first call on a device, with that device current, asks the runtime for
// the array's device address (hipGetSymbolAddress) and zeroes the array with a fill kernel; later
// calls on that device use the stored address. Every launch leaves the array zeroed again (the
// finishing workgroup clears what it used), so each call starts from zeros; calls that overlap on
// one GPU share the array and race.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "kohler.h"
#include "kohler_host.h"
#include "kohler_impl.h"

using namespace kohler;

namespace {

// int64 words: the accumulator replicas first, then the ticket and the range flag (two words).
constexpr int64_t kScratchAccWords = KOHLER_NOALLOC_SCRATCH_WORDS;
constexpr int64_t kScratchWords = kScratchAccWords + 2;
__device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned long long *g_ptr[kMaxDevices];  // device address of `scratch` per device, once known
int g_cus[kMaxDevices];

__global__ void zero_scratch(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// The scratch address and compute-unit count of the current device, set up on its first call.
int device_scratch(hipStream_t stream, unsigned long long **ptr, int *num_cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pick_status(e);
    if (dev < 0 || dev >= kMaxDevices) return KOHLER_E_DEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return pick_status(e);
        int cus = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return pick_status(e);
        hipLaunchKernelGGL(zero_scratch, dim3(64), dim3(256), 0, stream, static_cast<unsigned long long *>(p),
                           kScratchWords);
        if ((e = hipGetLastError()) != hipSuccess) return pick_status(e);
        g_ptr[dev] = static_cast<unsigned long long *>(p);
        g_cus[dev] = cus > 0 ? cus : 1;
    }
    *ptr = g_ptr[dev];
    *num_cus = g_cus[dev];
    return KOHLER_OK;
}

}  // namespace

extern "C" int kohler_curve_noalloc(const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                                    int32_t M, int32_t nbhd, int64_t *d_sum, int64_t *d_count, double *d_C,
                                    int32_t *d_thr, int32_t thr_capacity, int32_t *d_n_thr, int32_t *d_t0,
                                    int32_t *d_status, const kohler_plan *plan, kohler_stream_t stream) {
    if (!d_img || !valid_shape(dtype, H, W, pitch, M, nbhd)) return KOHLER_E_ARG;
    if (!d_sum || !d_count || !d_C || !d_n_thr || !d_t0 || !d_status) return KOHLER_E_ARG;
    if (thr_capacity < 0 || (thr_capacity > 0 && !d_thr)) return KOHLER_E_ARG;
    const int64_t rstride = replica_stride(M);
    if (rstride > kScratchAccWords) return KOHLER_E_ARG;  // more grey levels than the scratch holds

    kohler_plan pl = plan ? *plan : default_plan(dtype, M);
    if (pl.form == 0) {
        const kohler_plan d = default_plan(dtype, M);
        pl.form = d.form;
        if (pl.band == 0) pl.band = d.band;
    }
    if ((pl.form == FORM_MARG || pl.form == FORM_TRI) && pl.band == 0) pl.band = 1;
    if (pl.copies == 0) pl.copies = pl.form == FORM_BAND ? 2 : 1;
    if (!valid_plan(pl, dtype, M) || lds_bytes(pl.form, M, pl.band, pl.block, pl.copies) > kMaxLdsBytes ||
        pl.block > max_block_for(dtype, nbhd, pl.form, pl.px_per_lane, M))
        return KOHLER_E_ARG;

    unsigned long long *sc = nullptr;
    int num_cus = 1;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int st = device_scratch(s, &sc, &num_cus);
    if (st != KOHLER_OK) return st;

    const int64_t units = strips_of(W, pl.px_per_lane) * H;
    if (pl.grid == 0) {
        const int per_cu = blocks_per_cu(dtype, nbhd, pl.form, pl.px_per_lane, M, pl.band, pl.block, pl.copies);
        const int64_t waves = pl.block / 64;
        const int64_t want = (units + waves * 4 - 1) / (waves * 4);
        pl.grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)num_cus * per_cu));
    }
    pl.grid = std::max(pl.grid, min_grid_for(pl, nbhd, units));
    // replicas: the plan's (or about one per 32 workgroups), as many as the scratch holds
    int nrep = pl.replicas > 0 ? pl.replicas : replicas_for(pl.grid);
    nrep = (int)std::max<int64_t>(1, std::min<int64_t>(nrep, kScratchAccWords / rstride));

    KParams p{};
    p.img0 = describe(d_img, dtype, H, W, pitch, pl.px_per_lane, 0);
    p.n = 1;
    p.M = M;
    p.band = pl.band;
    p.copies = pl.copies;
    p.cap = thr_capacity;
    p.packed_acc = (!pl.acc_split && packable(H, W, nbhd)) ? 1 : 0;
    p.nrep = nrep;
    p.rep_stride = rstride;
    p.acc_stride = (int64_t)nrep * rstride;
    p.total_units = p.img0.nunits;
    p.acc = reinterpret_cast<int64_t *>(sc);
    p.done = sc + kScratchAccWords;
    p.rflag = reinterpret_cast<uint32_t *>(sc + kScratchAccWords + 1);
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
    return pick_status(launch_curve(p, dtype, nbhd, pl.form, pl.px_per_lane, pl.block, pl.grid, s));
}
