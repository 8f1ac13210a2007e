// Consumers of the contrast curve's thresholds (G. Noyel, arXiv 1707.05062, Sec. 2.1): the lower set
// of a threshold t is {f <= t} (eq (1)), so ascending thresholds t_1 < ... < t_k cut the grey levels
// into k + 1 classes, and a pixel of value f is in class #{i : t_i < f}. Each class of the paper's
// Fig. 1 is shown at the mean value of its pixels, and its thresholds are the most significant
// maxima of the curve.
//
//   segment_kernel     labels (or class means) of every pixel: a stream over the image; every
//                      workgroup first builds a table for the M + 1 grey levels in LDS (one binary
//                      search per level over the thresholds in LDS; level M stands for every value
//                      >= M), then maps pixels through it, 16 bytes of input per lane and step, with
//                      loads of several steps in flight. Each pixel is read once and written once.
//   class_stats_kernel the image's grey-level histogram (same stream shape, LDS counters per
//                      workgroup, one global atomic per non-empty level and workgroup), folded
//                      into per-class count, sum and mean by the workgroup that finishes last,
//                      which also clears the histogram for the next call
//   top_kernel         one workgroup: the k thresholds of largest C, by exact rank
//
// The entry points (kohler_segment, kohler_class_stats, kohler_mean_image, kohler_top_thresholds) are
// declared in include/kohler.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kohler.h"
#include "kohler_host.h"

namespace kohler {
namespace {

#define KOHLER_SEG_GLOBAL __attribute__((address_space(1)))
#define KOHLER_SEG_LDS __attribute__((address_space(3)))

constexpr int kSegBlock = 256;
constexpr int kSegUnroll = 4;  // 16-byte input groups a lane has in flight per step

struct SegParams {
    const void *img;
    int64_t H, W, pitch;
    void *out;
    int64_t out_pitch;
    const int32_t *thr;
    const int32_t *n_thr;
    int32_t M, cap;
    int32_t flat;    // 1: input and output rows are contiguous (pitch == W) and 16-byte aligned
    int32_t copies;  // histogram: LDS copies of each counter (a power of two), lane l uses copy l mod copies
    const double *mean;  // non-null: the table holds each class's rounded mean instead of its label
};

typedef uint32_t seg_u32x4 __attribute__((ext_vector_type(4)));

template <typename Pout>
__device__ __forceinline__ uint32_t lut_of(const KOHLER_SEG_LDS Pout *lut, uint32_t v, uint32_t Mtop) {
    return (uint32_t)lut[min(v, Mtop)];  // entry M stands for every value >= M
}

// Number of thresholds below v among the n ascending ones at thr (first index with thr[i] >= v).
template <class T>
__device__ __forceinline__ int rank_below(const T *thr, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (thr[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Labels of the 16 input bytes of one group, packed as the output row holds them.
template <typename Pin, typename Pout>
__device__ __forceinline__ void map_group(const seg_u32x4 in, const KOHLER_SEG_LDS Pout *lut, uint32_t Mtop,
                                          Pout (&o)[16 / sizeof(Pin)]) {
    constexpr int PPW = 4 / (int)sizeof(Pin);  // pixels per input word
    constexpr uint32_t MASK = sizeof(Pin) == 1 ? 0xFFu : 0xFFFFu;
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int k = 0; k < PPW; ++k) o[w * PPW + k] = (Pout)lut_of(lut, (in[w] >> (8 * (int)sizeof(Pin) * k)) & MASK, Mtop);
}

template <typename Pin, typename Pout>
__global__ void __launch_bounds__(kSegBlock) segment_kernel(SegParams p) {
    extern __shared__ __align__(16) uint8_t seg_lds[];
    KOHLER_SEG_LDS uint8_t *lbase = (KOHLER_SEG_LDS uint8_t *)seg_lds;
    KOHLER_SEG_LDS Pout *lut = reinterpret_cast<KOHLER_SEG_LDS Pout *>(lbase);  // M labels
    KOHLER_SEG_LDS int32_t *thr = reinterpret_cast<KOHLER_SEG_LDS int32_t *>(
        lbase + (((size_t)(p.M + 1) * sizeof(Pout) + 15) & ~(size_t)15));  // cap

    const int n = min(max(*p.n_thr, 0), p.cap);  // thresholds in use (a capacity-truncated list too)
    for (int i = threadIdx.x; i < n; i += blockDim.x) thr[i] = p.thr[i];
    __syncthreads();
    for (int v = threadIdx.x; v <= p.M; v += blockDim.x) {
        const int j = rank_below(thr, n, v);
        lut[v] = p.mean ? (Pout)__builtin_rint(p.mean[j]) : (Pout)j;  // ties to even
    }
    __syncthreads();
    const uint32_t Mtop = (uint32_t)p.M;  // index of the table's last entry

    if (p.flat) {
        // the image as one array of N pixels, in 16-byte groups of G pixels
        constexpr int G = 16 / (int)sizeof(Pin);
        const int64_t N = p.H * p.W;
        const int64_t ngroups = N / G;
        const KOHLER_SEG_GLOBAL seg_u32x4 *src = (const KOHLER_SEG_GLOBAL seg_u32x4 *)p.img;
        KOHLER_SEG_GLOBAL Pout *dst = (KOHLER_SEG_GLOBAL Pout *)p.out;
        const int64_t span = (int64_t)gridDim.x * kSegBlock * kSegUnroll;
        for (int64_t g0 = (int64_t)blockIdx.x * kSegBlock * kSegUnroll + threadIdx.x; g0 < ngroups; g0 += span) {
            seg_u32x4 in[kSegUnroll];
#pragma unroll
            for (int u = 0; u < kSegUnroll; ++u) {
                const int64_t g = g0 + (int64_t)u * kSegBlock;
                in[u] = src[min(g, ngroups - 1)];  // unconditional: the surplus re-reads the last group
            }
#pragma unroll
            for (int u = 0; u < kSegUnroll; ++u) {
                const int64_t g = g0 + (int64_t)u * kSegBlock;
                if (g < ngroups) {
                    Pout o[G];
                    map_group<Pin, Pout>(in[u], lut, Mtop, o);
                    // G labels, packed into NW 32-bit words: 32, 16 or 8 bytes per group
                    constexpr int LPW = 4 / (int)sizeof(Pout);
                    constexpr int NW = G / LPW;
                    uint32_t w[NW];
#pragma unroll
                    for (int k = 0; k < NW; ++k) {
                        uint32_t x = 0;
#pragma unroll
                        for (int b = 0; b < LPW; ++b) x |= (uint32_t)o[k * LPW + b] << (8 * (int)sizeof(Pout) * b);
                        w[k] = x;
                    }
                    KOHLER_SEG_GLOBAL uint32_t *dw = reinterpret_cast<KOHLER_SEG_GLOBAL uint32_t *>(dst + g * G);
                    if constexpr (NW >= 4) {
#pragma unroll
                        for (int k = 0; k < NW; k += 4)
                            *reinterpret_cast<KOHLER_SEG_GLOBAL seg_u32x4 *>(dw + k) = seg_u32x4{w[k], w[k + 1], w[k + 2], w[k + 3]};
                    } else {
                        typedef uint32_t seg_u32x2 __attribute__((ext_vector_type(2)));
                        *reinterpret_cast<KOHLER_SEG_GLOBAL seg_u32x2 *>(dw) = seg_u32x2{w[0], w[1]};
                    }
                }
            }
        }
        // the last N mod G pixels
        const int64_t tail = ngroups * G;
        const KOHLER_SEG_GLOBAL Pin *s1 = (const KOHLER_SEG_GLOBAL Pin *)p.img;
        for (int64_t i = tail + (int64_t)blockIdx.x * kSegBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kSegBlock)
            dst[i] = (Pout)lut_of(lut, (uint32_t)s1[i], Mtop);
    } else {
        // rows with a pitch: one pixel per lane and step
        const KOHLER_SEG_GLOBAL Pin *src = (const KOHLER_SEG_GLOBAL Pin *)p.img;
        KOHLER_SEG_GLOBAL Pout *dst = (KOHLER_SEG_GLOBAL Pout *)p.out;
        for (int64_t r = blockIdx.x; r < p.H; r += gridDim.x)
            for (int64_t c = threadIdx.x; c < p.W; c += kSegBlock)
                dst[r * p.out_pitch + c] = (Pout)lut_of(lut, (uint32_t)src[r * p.pitch + c], Mtop);
    }
}

// Memory shared between the workgroups of the class-statistics launch (histogram, ticket) is only
// touched with system-scope atomics, which are performed past the per-XCD L2 caches: a workgroup's
// additions are complete once their returned values have arrived, so the workgroup that takes the
// last ticket sees every addition without a device-wide cache flush.
#define KOHLER_SEG_XSCOPE __HIP_MEMORY_SCOPE_SYSTEM

constexpr int kHistBlock = 1024;

// Per-class count, value sum and mean for class j = levels v with #{i : t_i < v} = j, from the
// histogram (level M holds the values >= M, counted at the value M), by the workgroup that took the
// last ticket; the class accumulators live in LDS (cap + 1 pairs of 64-bit words). Clears the
// histogram and the ticket for the next call.
__device__ void fold_classes(const SegParams &p, unsigned long long *hist, unsigned long long *ticket,
                             int64_t *count, int64_t *sum, double *mean, KOHLER_SEG_LDS uint8_t *lds) {
    KOHLER_SEG_LDS unsigned long long *ck = (KOHLER_SEG_LDS unsigned long long *)lds;  // cap + 1
    KOHLER_SEG_LDS unsigned long long *cs = ck + (p.cap + 1);                           // cap + 1
    KOHLER_SEG_LDS int32_t *thr = (KOHLER_SEG_LDS int32_t *)(cs + (p.cap + 1));         // cap
    const int n = min(max(*p.n_thr, 0), p.cap);
    for (int j = threadIdx.x; j <= p.cap; j += blockDim.x) ck[j] = cs[j] = 0ull;
    for (int i = threadIdx.x; i < n; i += blockDim.x) thr[i] = p.thr[i];
    __syncthreads();
    for (int v = threadIdx.x; v <= p.M; v += blockDim.x) {
        const unsigned long long c = __hip_atomic_load(hist + v, __ATOMIC_RELAXED, KOHLER_SEG_XSCOPE);
        if (c) {
            const int j = rank_below(thr, n, v);
            __hip_atomic_fetch_add(ck + j, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(cs + j, c * (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(hist + v, 0ull, __ATOMIC_RELAXED, KOHLER_SEG_XSCOPE);
        }
    }
    if (threadIdx.x == 0) __hip_atomic_store(ticket, 0ull, __ATOMIC_RELAXED, KOHLER_SEG_XSCOPE);
    __syncthreads();
    for (int j = threadIdx.x; j <= p.cap; j += blockDim.x) {
        const int64_t c = j <= n ? (int64_t)ck[j] : 0, s = j <= n ? (int64_t)cs[j] : 0;
        count[j] = c;
        sum[j] = s;
        mean[j] = c ? (double)s / (double)c : 0.0;  // one correctly rounded division
    }
}

// Class statistics in one launch. Every workgroup counts its share of the pixels into LDS counters
// (32 bits: a workgroup sees fewer than 2^32 pixels), `copies` of each level side by side so that
// lanes of one wave counting the same grey level (flat regions) mostly hit different words, adds
// its non-empty levels to hist[0..M] (entry M counts every value >= M), then takes a ticket; the
// last workgroup folds the histogram into the classes.

template <typename Pin>
__global__ void __launch_bounds__(kHistBlock) class_stats_kernel(SegParams p, unsigned long long *hist,
                                                                  unsigned long long *ticket, int64_t *out_count,
                                                                  int64_t *out_sum, double *out_mean) {
    extern __shared__ __align__(16) uint8_t seg_lds[];
    KOHLER_SEG_LDS uint32_t *h = (KOHLER_SEG_LDS uint32_t *)seg_lds;  // (M + 1) * copies counters
    const uint32_t nc = (uint32_t)p.copies;
    for (uint32_t x = threadIdx.x; x < ((uint32_t)p.M + 1u) * nc; x += blockDim.x) h[x] = 0u;
    __syncthreads();
    const uint32_t Mtop = (uint32_t)p.M;
    KOHLER_SEG_LDS uint32_t *hl = h + (threadIdx.x & (nc - 1u));
    auto count = [&](uint32_t v) {
        __hip_atomic_fetch_add(hl + min(v, Mtop) * nc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    if (p.flat) {
        constexpr int G = 16 / (int)sizeof(Pin);
        constexpr int PPW = 4 / (int)sizeof(Pin);
        constexpr uint32_t MASK = sizeof(Pin) == 1 ? 0xFFu : 0xFFFFu;
        const int64_t N = p.H * p.W;
        const int64_t ngroups = N / G;
        const KOHLER_SEG_GLOBAL seg_u32x4 *src = (const KOHLER_SEG_GLOBAL seg_u32x4 *)p.img;
        const int64_t span = (int64_t)gridDim.x * kHistBlock * kSegUnroll;
        for (int64_t g0 = (int64_t)blockIdx.x * kHistBlock * kSegUnroll + threadIdx.x; g0 < ngroups; g0 += span) {
            seg_u32x4 in[kSegUnroll];
#pragma unroll
            for (int u = 0; u < kSegUnroll; ++u) in[u] = src[min(g0 + (int64_t)u * kHistBlock, ngroups - 1)];
#pragma unroll
            for (int u = 0; u < kSegUnroll; ++u) {
                if (g0 + (int64_t)u * kHistBlock < ngroups) {
#pragma unroll
                    for (int w = 0; w < 4; ++w)
#pragma unroll
                        for (int k = 0; k < PPW; ++k) count((in[u][w] >> (8 * (int)sizeof(Pin) * k)) & MASK);
                }
            }
        }
        const KOHLER_SEG_GLOBAL Pin *s1 = (const KOHLER_SEG_GLOBAL Pin *)p.img;
        for (int64_t i = ngroups * G + (int64_t)blockIdx.x * kHistBlock + threadIdx.x; i < N;
             i += (int64_t)gridDim.x * kHistBlock)
            count((uint32_t)s1[i]);
    } else {
        const KOHLER_SEG_GLOBAL Pin *src = (const KOHLER_SEG_GLOBAL Pin *)p.img;
        for (int64_t r = blockIdx.x; r < p.H; r += gridDim.x)
            for (int64_t c = threadIdx.x; c < p.W; c += kHistBlock) count((uint32_t)src[r * p.pitch + c]);
    }
    __syncthreads();
    uint64_t sink = 0;
    for (int v = threadIdx.x; v <= p.M; v += blockDim.x) {
        unsigned long long c = 0;
        for (uint32_t k = 0; k < nc; ++k) c += h[(uint32_t)v * nc + k];
        if (c) sink ^= __hip_atomic_fetch_add(hist + v, c, __ATOMIC_RELAXED, KOHLER_SEG_XSCOPE);
    }
    // consuming the returned values makes the wave wait until its additions are performed
    asm volatile("" ::"v"((uint32_t)sink), "v"((uint32_t)(sink >> 32)));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    KOHLER_SEG_LDS uint32_t *last = h;  // the counters are dead now
    if (threadIdx.x == 0) {
        const unsigned long long old = __hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, KOHLER_SEG_XSCOPE);
        *last = (old + 1ull == (unsigned long long)gridDim.x) ? 1u : 0u;
    }
    __syncthreads();
    const bool is_last = *last != 0u;
    __syncthreads();  // every thread has read the flag before the fold reuses the LDS
    if (is_last) fold_classes(p, hist, ticket, out_count, out_sum, out_mean, (KOHLER_SEG_LDS uint8_t *)seg_lds);
}

constexpr int kOneBlock = 1024;
constexpr int kHistCopies = 8;

// sign(C(u) - C(v)) exactly for C = s / k (0 when k == 0), s, k >= 0: 128-bit cross products.
__device__ __forceinline__ int cmp_ratio(int64_t su, int64_t ku, int64_t sv, int64_t kv) {
    const uint64_t nu = ku ? (uint64_t)su : 0, du = ku ? (uint64_t)ku : 1;
    const uint64_t nv = kv ? (uint64_t)sv : 0, dv = kv ? (uint64_t)kv : 1;
    const uint64_t lh = __umul64hi(nu, dv), ll = nu * dv;
    const uint64_t rh = __umul64hi(nv, du), rl = nv * du;
    if (lh != rh) return lh > rh ? 1 : -1;
    if (ll != rl) return ll > rl ? 1 : -1;
    return 0;
}

struct TopParams {
    const int64_t *sum, *count;
    const int32_t *thr, *n_thr;
    int32_t *top, *n_top;
    int32_t M, cap, k, pad;
};

// The k thresholds of largest C, largest first, equal C in ascending t. Every threshold's place in
// that order is its exact rank (the number of thresholds before it), so the ranks below k are the
// output slots. Thresholds outside [0, M) count as C = 0. One workgroup.
__global__ void __launch_bounds__(kOneBlock) top_kernel(TopParams p) {
    const int n = min(max(*p.n_thr, 0), p.cap);
    const int kk = min(p.k, n);
    auto load = [&](int i, int32_t &t, int64_t &s, int64_t &c) {
        t = p.thr[i];
        const bool ok = t >= 0 && t < p.M;
        s = ok ? p.sum[t] : 0;
        c = ok ? p.count[t] : 0;
    };
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        int32_t ti;
        int64_t si, ci;
        load(i, ti, si, ci);
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            int32_t tj;
            int64_t sj, cj;
            load(j, tj, sj, cj);
            const int r = cmp_ratio(sj, cj, si, ci);
            rank += (r > 0 || (r == 0 && tj < ti)) ? 1 : 0;
        }
        if (rank < kk) p.top[rank] = ti;
    }
    if (threadIdx.x == 0) *p.n_top = kk;
}

const void *seg_kernel_for(int dtype, int label_dtype) {
    if (dtype == KOHLER_U8)
        return label_dtype == KOHLER_U8 ? reinterpret_cast<const void *>(segment_kernel<uint8_t, uint8_t>)
                                        : reinterpret_cast<const void *>(segment_kernel<uint8_t, uint16_t>);
    return label_dtype == KOHLER_U8 ? reinterpret_cast<const void *>(segment_kernel<uint16_t, uint8_t>)
                                    : reinterpret_cast<const void *>(segment_kernel<uint16_t, uint16_t>);
}

// Two classes at the image's own t0 (read from device memory): blockIdx.y picks the image; each
// lane labels 4 consecutive pixels of a row per step, the workgroups striding over the rows.
template <typename Pin>
__global__ void __launch_bounds__(kSegBlock) label_t0_kernel(LabelJobs js) {
    const LabelJob &jb = js.job[blockIdx.y];
    const int32_t t0 = *(const KOHLER_SEG_GLOBAL int32_t *)jb.t0;
    const int64_t quads = (jb.W + 3) / 4;
    const int64_t total = jb.H * quads;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = q / quads, x0 = (q - y * quads) * 4;
        const KOHLER_SEG_GLOBAL Pin *row = (const KOHLER_SEG_GLOBAL Pin *)(static_cast<const Pin *>(jb.img) + y * jb.pitch);
        KOHLER_SEG_GLOBAL uint8_t *out = (KOHLER_SEG_GLOBAL uint8_t *)(jb.labels + y * jb.lpitch);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (x0 + k < jb.W) out[x0 + k] = (t0 >= 0 && (int32_t)row[x0 + k] > t0) ? 1 : 0;
    }
}

}  // namespace

hipError_t launch_label_t0(const LabelJobs &js, hipStream_t stream) {
    if (js.n < 1 || js.n > kMaxLabelJobs) return hipErrorInvalidValue;
    int64_t most = 1;
    for (int i = 0; i < js.n; ++i) most = std::max<int64_t>(most, js.job[i].H * ((js.job[i].W + 3) / 4));
    const int gx = (int)std::min<int64_t>((most + kSegBlock - 1) / kSegBlock, 1024);
    LabelJobs arg = js;
    void *args[] = {&arg};
    const void *kern = js.dtype == KOHLER_U8 ? reinterpret_cast<const void *>(label_t0_kernel<uint8_t>)
                                             : reinterpret_cast<const void *>(label_t0_kernel<uint16_t>);
    hipError_t e = hipLaunchKernel(kern, dim3(gx, js.n), dim3(kSegBlock), args, 0, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace kohler

using namespace kohler;

namespace {

int64_t stream_grid(kohler_ctx *ctx, const SegParams &p, int dtype) {
    // enough workgroups to keep every compute unit streaming, no more than the work needs
    const int64_t esz = dtype == KOHLER_U8 ? 1 : 2;
    const int64_t per_block = (int64_t)kSegBlock * kSegUnroll * (16 / esz);
    const int64_t want = p.flat ? (p.H * p.W + per_block - 1) / per_block : p.H;
    return std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * 8));
}

int launch(const void *kern, int grid, int block, void **args, size_t lds, kohler_stream_t stream) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, lds, stream);
    if (e == hipSuccess) e = hipGetLastError();
    return pick_status(e);
}

SegParams seg_params(const void *d_img, int64_t H, int64_t W, int64_t pitch, int32_t M, const int32_t *d_thr,
                     const int32_t *d_n_thr, int32_t cap, void *d_out, int64_t out_pitch) {
    SegParams p{};
    p.img = d_img;
    p.H = H;
    p.W = W;
    p.pitch = pitch;
    p.out = d_out;
    p.out_pitch = out_pitch;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.M = M;
    p.cap = cap;
    const bool out_flat = !d_out || (out_pitch == W && reinterpret_cast<uintptr_t>(d_out) % 16 == 0);
    p.flat = (pitch == W && reinterpret_cast<uintptr_t>(d_img) % 16 == 0 && out_flat) ? 1 : 0;
    return p;
}

// Table (M + 1 entries of the output type) and thresholds in LDS, then the pixel stream.
int launch_map(kohler_ctx *ctx, const SegParams &p0, int dtype, int out_dtype, kohler_stream_t stream) {
    SegParams p = p0;
    const size_t osz = out_dtype == KOHLER_U8 ? 1 : 2;
    const size_t lds = (((size_t)(p.M + 1) * osz + 15) & ~(size_t)15) + 4 * (size_t)std::max(p.cap, 1);
    void *args[] = {&p};
    return launch(seg_kernel_for(dtype, out_dtype), (int)stream_grid(ctx, p, dtype), kSegBlock, args, lds, stream);
}

bool common_args(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch, int32_t M,
                 const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity) {
    if (!ctx || !d_img || !d_n_thr) return false;
    if (!valid_shape(dtype, H, W, pitch, M, 4)) return false;
    return thr_capacity >= 0 && thr_capacity <= M && (thr_capacity == 0 || d_thr);
}

}  // namespace

extern "C" int kohler_segment(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                              int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                              void *d_labels, int label_dtype, int64_t label_pitch, kohler_stream_t stream) {
    if (!common_args(ctx, d_img, dtype, H, W, pitch, M, d_thr, d_n_thr, thr_capacity) || !d_labels) return KOHLER_E_ARG;
    if (label_dtype != KOHLER_U8 && label_dtype != KOHLER_U16) return KOHLER_E_ARG;
    if (label_pitch < W) return KOHLER_E_ARG;
    if (label_dtype == KOHLER_U8 && thr_capacity > 255) return KOHLER_E_ARG;  // labels up to the capacity
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    const SegParams p = seg_params(d_img, H, W, pitch, M, d_thr, d_n_thr, thr_capacity, d_labels, label_pitch);
    return launch_map(ctx, p, dtype, label_dtype, stream);
}

extern "C" int kohler_mean_image(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                                 int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                                 const double *d_mean, void *d_out, int64_t out_pitch, kohler_stream_t stream) {
    if (!common_args(ctx, d_img, dtype, H, W, pitch, M, d_thr, d_n_thr, thr_capacity) || !d_mean || !d_out)
        return KOHLER_E_ARG;
    if (out_pitch < W) return KOHLER_E_ARG;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    SegParams p = seg_params(d_img, H, W, pitch, M, d_thr, d_n_thr, thr_capacity, d_out, out_pitch);
    p.mean = d_mean;
    return launch_map(ctx, p, dtype, dtype, stream);  // the output has the image's type
}

extern "C" int kohler_class_stats(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                                  int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                                  int64_t *d_count, int64_t *d_sum, double *d_mean, kohler_stream_t stream) {
    if (!common_args(ctx, d_img, dtype, H, W, pitch, M, d_thr, d_n_thr, thr_capacity)) return KOHLER_E_ARG;
    if (!d_count || !d_sum || !d_mean || thr_capacity > KOHLER_MAX_CLASS_THRESHOLDS) return KOHLER_E_ARG;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    unsigned long long *hist = nullptr;
    {
        // the histogram scratch: M + 1 words for the largest M, zero between calls
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!ctx->level_hist) {
            void *q = nullptr;
            const size_t bytes = sizeof(unsigned long long) * ((size_t)kMaxM + 2);  // histogram, ticket
            if ((e = hipMalloc(&q, bytes)) != hipSuccess) return pick_status(e);
            if ((e = hipMemset(q, 0, bytes)) != hipSuccess) {
                (void)hipFree(q);
                return pick_status(e);
            }
            ctx->level_hist = static_cast<unsigned long long *>(q);
        }
        hist = ctx->level_hist;
    }
    SegParams p = seg_params(d_img, H, W, pitch, M, d_thr, d_n_thr, thr_capacity, nullptr, 0);
    // as many counter copies as fit in 32 KiB of LDS (at most kHistCopies), and two 1024-thread
    // workgroups per compute unit: each streams a large share, and few partial histograms meet in
    // the atomics
    p.copies = 1;
    while (p.copies < kHistCopies && 4 * ((size_t)M + 1) * (size_t)(2 * p.copies) <= 32768) p.copies *= 2;
    unsigned long long *ticket = hist + (kMaxM + 1);
    void *args[] = {&p, &hist, &ticket, &d_count, &d_sum, &d_mean};
    const void *hk = dtype == KOHLER_U8 ? reinterpret_cast<const void *>(class_stats_kernel<uint8_t>)
                                        : reinterpret_cast<const void *>(class_stats_kernel<uint16_t>);
    const int64_t per_block = (int64_t)kHistBlock * kSegUnroll * (dtype == KOHLER_U8 ? 16 : 8);
    const int64_t want = p.flat ? (H * W + per_block - 1) / per_block : H;
    const int hgrid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * 2));
    const size_t lds = std::max(4 * ((size_t)M + 1) * (size_t)p.copies,
                                16 * ((size_t)thr_capacity + 1) + 4 * (size_t)std::max(thr_capacity, 1));
    return launch(hk, hgrid, kHistBlock, args, lds, stream);
}

extern "C" int kohler_top_thresholds(kohler_ctx *ctx, const int64_t *d_sum, const int64_t *d_count, int32_t M,
                                     const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity, int32_t k,
                                     int32_t *d_top, int32_t *d_n_top, kohler_stream_t stream) {
    if (!ctx || !d_sum || !d_count || !d_n_thr || !d_n_top || M < 1 || k < 0) return KOHLER_E_ARG;
    if (thr_capacity < 0 || thr_capacity > M || (thr_capacity > 0 && !d_thr) || (k > 0 && !d_top)) return KOHLER_E_ARG;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);
    TopParams p{d_sum, d_count, d_thr, d_n_thr, d_top, d_n_top, M, thr_capacity, k, 0};
    void *args[] = {&p};
    return launch(reinterpret_cast<const void *>(top_kernel), 1, kOneBlock, args, 0, stream);
}
