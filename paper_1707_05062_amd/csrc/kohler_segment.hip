// Segmentation by the thresholds of the contrast curve (G. Noyel, arXiv 1707.05062, Sec. 2.1): the
// lower set of a threshold t is {f <= t} (eq (1)), so ascending thresholds t_1 < ... < t_k cut the
// grey levels into k + 1 classes, and a pixel of value f is labelled #{i : t_i < f}.
//
// The kernel is a stream over the image: every workgroup first builds a label table for the M grey
// levels in LDS (thresholds copied to LDS, one binary search per level), then maps pixels through it,
// 16 bytes of input per lane and step, with loads of several steps in flight. Each pixel is read
// once and its label written once; the entry point kohler_segment is declared in include/kohler.h.

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
    int32_t flat;  // 1: input and output rows are contiguous (pitch == W) and 16-byte aligned
    int32_t pad;
};

typedef uint32_t seg_u32x4 __attribute__((ext_vector_type(4)));

template <typename Pout>
__device__ __forceinline__ uint32_t lut_of(const KOHLER_SEG_LDS Pout *lut, uint32_t v, uint32_t Mm1) {
    return (uint32_t)lut[min(v, Mm1)];  // values past M - 1 take the top level's label
}

// Labels of the 16 input bytes of one group, packed as the output row holds them.
template <typename Pin, typename Pout>
__device__ __forceinline__ void map_group(const seg_u32x4 in, const KOHLER_SEG_LDS Pout *lut, uint32_t Mm1,
                                          Pout (&o)[16 / sizeof(Pin)]) {
    constexpr int PPW = 4 / (int)sizeof(Pin);  // pixels per input word
    constexpr uint32_t MASK = sizeof(Pin) == 1 ? 0xFFu : 0xFFFFu;
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int k = 0; k < PPW; ++k) o[w * PPW + k] = (Pout)lut_of(lut, (in[w] >> (8 * (int)sizeof(Pin) * k)) & MASK, Mm1);
}

template <typename Pin, typename Pout>
__global__ void __launch_bounds__(kSegBlock) segment_kernel(SegParams p) {
    extern __shared__ __align__(16) uint8_t seg_lds[];
    KOHLER_SEG_LDS uint8_t *lbase = (KOHLER_SEG_LDS uint8_t *)seg_lds;
    KOHLER_SEG_LDS Pout *lut = reinterpret_cast<KOHLER_SEG_LDS Pout *>(lbase);  // M labels
    KOHLER_SEG_LDS int32_t *thr =
        reinterpret_cast<KOHLER_SEG_LDS int32_t *>(lbase + ((p.M * sizeof(Pout) + 15) & ~(size_t)15));  // cap

    const int n = min(max(*p.n_thr, 0), p.cap);  // thresholds in use (a capacity-truncated list too)
    for (int i = threadIdx.x; i < n; i += blockDim.x) thr[i] = p.thr[i];
    __syncthreads();
    for (int v = threadIdx.x; v < p.M; v += blockDim.x) {
        int lo = 0, hi = n;  // number of thresholds below v: first index with thr[i] >= v
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (thr[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        lut[v] = (Pout)lo;
    }
    __syncthreads();
    const uint32_t Mm1 = (uint32_t)p.M - 1u;

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
                    map_group<Pin, Pout>(in[u], lut, Mm1, o);
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
            dst[i] = (Pout)lut_of(lut, (uint32_t)s1[i], Mm1);
    } else {
        // rows with a pitch: one pixel per lane and step
        const KOHLER_SEG_GLOBAL Pin *src = (const KOHLER_SEG_GLOBAL Pin *)p.img;
        KOHLER_SEG_GLOBAL Pout *dst = (KOHLER_SEG_GLOBAL Pout *)p.out;
        for (int64_t r = blockIdx.x; r < p.H; r += gridDim.x)
            for (int64_t c = threadIdx.x; c < p.W; c += kSegBlock)
                dst[r * p.out_pitch + c] = (Pout)lut_of(lut, (uint32_t)src[r * p.pitch + c], Mm1);
    }
}

const void *seg_kernel_for(int dtype, int label_dtype) {
    if (dtype == KOHLER_U8)
        return label_dtype == KOHLER_U8 ? reinterpret_cast<const void *>(segment_kernel<uint8_t, uint8_t>)
                                        : reinterpret_cast<const void *>(segment_kernel<uint8_t, uint16_t>);
    return label_dtype == KOHLER_U8 ? reinterpret_cast<const void *>(segment_kernel<uint16_t, uint8_t>)
                                    : reinterpret_cast<const void *>(segment_kernel<uint16_t, uint16_t>);
}

}  // namespace
}  // namespace kohler

using namespace kohler;

extern "C" int kohler_segment(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                              int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                              void *d_labels, int label_dtype, int64_t label_pitch, kohler_stream_t stream) {
    if (!ctx || !d_img || !d_n_thr || !d_labels) return KOHLER_E_ARG;
    if (!valid_shape(dtype, H, W, pitch, M, 4)) return KOHLER_E_ARG;
    if (label_dtype != KOHLER_U8 && label_dtype != KOHLER_U16) return KOHLER_E_ARG;
    if (label_pitch < W || thr_capacity < 0 || thr_capacity > M || (thr_capacity > 0 && !d_thr)) return KOHLER_E_ARG;
    if (label_dtype == KOHLER_U8 && thr_capacity > 255) return KOHLER_E_ARG;  // labels up to the capacity
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return pick_status(e);

    SegParams p{};
    p.img = d_img;
    p.H = H;
    p.W = W;
    p.pitch = pitch;
    p.out = d_labels;
    p.out_pitch = label_pitch;
    p.thr = d_thr;
    p.n_thr = d_n_thr;
    p.M = M;
    p.cap = thr_capacity;
    p.flat = (pitch == W && label_pitch == W && reinterpret_cast<uintptr_t>(d_img) % 16 == 0 &&
              reinterpret_cast<uintptr_t>(d_labels) % 16 == 0) ? 1 : 0;
    const size_t osz = label_dtype == KOHLER_U8 ? 1 : 2;
    const size_t lds = (((size_t)M * osz + 15) & ~(size_t)15) + 4 * (size_t)std::max(thr_capacity, 1);
    const void *kern = seg_kernel_for(dtype, label_dtype);
    if ((e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
        return pick_status(e);
    // enough workgroups to keep every compute unit streaming, no more than the work needs
    const int64_t esz = dtype == KOHLER_U8 ? 1 : 2;
    const int64_t per_block = (int64_t)kSegBlock * kSegUnroll * (16 / esz);
    const int64_t want = p.flat ? (H * W + per_block - 1) / per_block : H;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)ctx->num_cus * 8));
    void *args[] = {&p};
    e = hipLaunchKernel(kern, dim3(grid), dim3(kSegBlock), args, lds, stream);
    if (e == hipSuccess) e = hipGetLastError();
    return pick_status(e);
}
