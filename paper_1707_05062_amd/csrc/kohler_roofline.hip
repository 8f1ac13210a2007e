// Roofline probes for the curve kernel's two bounding resources on gfx950, built into
// libkohler_roofline.so and used by the benchmark only (not part of the curve library):
//   * the HBM read stream: every byte of a device buffer read once with 16-byte vector loads, the
//     rate the curve kernel's one pass over the image is compared with;
//   * LDS atomic increments (ds_add_u32 without return, as the curve kernel issues one per
//     neighbour pair) at several address patterns, the rate its pair phase is compared with.
// Each entry point only enqueues one launch on the given stream; the caller times it.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#define ROOF_GLOBAL __attribute__((address_space(1)))

// Reads n16 16-byte words; a thread keeps 4 loads in flight. The XOR of everything read is stored
// only if it equals a value the caller passes (never, in practice), so the loads stay live.
__global__ void __launch_bounds__(256) read_stream_kernel(const u32x4 *p, uint64_t n16, uint32_t never,
                                                          uint32_t *sink) {
    const ROOF_GLOBAL u32x4 *q = (const ROOF_GLOBAL u32x4 *)p;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = q[i], b = q[i + stride], c = q[i + 2 * stride], d = q[i + 3 * stride];
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < n16; i += stride) acc ^= q[i];
    const uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (x == never) sink[threadIdx.x & 63] = x;
}

// LDS address patterns (word indices into a table of 33 rows of kRowWords words, dynamic LDS):
enum Pattern : int {
    PAT_DISTINCT = 0,  // each lane of a wave its own consecutive word: no bank conflict, no collision
    PAT_RAND256 = 1,   // uniform over 256 words: collisions and bank conflicts of a 256-level histogram
    PAT_BAND = 2,      // uniform over a 33 x 257-word joint table (the banded (gap, low) histogram)
    PAT_SMOOTH = 3,    // joint-table words of a smooth image: gap 0..14 (triangular), low value within
                       // 16 of a level shared by the wave
    PAT_SAME = 4,      // every lane of a wave on one word
};
constexpr uint32_t kRowWords = 257;
constexpr int kUnroll = 16;

__device__ __forceinline__ uint32_t xorshift(uint32_t x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

// The table lives in dynamic LDS (after the one static word below) and its row length arrives as an
// argument, so every pattern keeps one address register per unrolled increment.
template <int PAT>
__global__ void __launch_bounds__(1024) lds_atomic_kernel(int iters, uint32_t seed, uint32_t *out,
                                                          uint32_t row_words) {
    extern __shared__ uint32_t tab[];
    const uint32_t table_words = 33u * row_words;
    for (uint32_t i = threadIdx.x; i < table_words; i += blockDim.x) tab[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = seed ^ (blockIdx.x * 0x9E3779B9u) ^ (threadIdx.x * 0x85EBCA6Bu) ^ 0x1234567u;
    uint32_t a[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
        x = xorshift(x);
        uint32_t w;
        if constexpr (PAT == PAT_DISTINCT) {
            w = (wave * 64u + lane + 1024u * (uint32_t)(k & 3)) % table_words;
        } else if constexpr (PAT == PAT_RAND256) {
            w = x & 255u;
        } else if constexpr (PAT == PAT_BAND) {
            w = (x >> 8) % table_words;
        } else if constexpr (PAT == PAT_SMOOTH) {
            const uint32_t centre = ((blockIdx.x * 7u + wave * 5u + (uint32_t)k * 13u) & 127u) + 32u;
            const uint32_t d = (x & 7u) + ((x >> 3) & 7u);
            w = d * row_words + centre + ((x >> 6) & 15u);
        } else {
            w = wave * 64u + (uint32_t)k;
        }
        a[k] = w;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k)
            __hip_atomic_fetch_add(&tab[a[k]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    uint32_t s = 0;
    for (uint32_t i = threadIdx.x; i < table_words; i += blockDim.x) s += tab[i];
    // the table total is blockDim * iters * kUnroll, added up per workgroup (so the atomics stay
    // live) through one LDS word and ONE global atomic: a global atomic per thread on the same
    // address would be serialised and take longer than the increments being measured
    __shared__ uint32_t total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    if (s) __hip_atomic_fetch_add(&total, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = total;
}

}  // namespace

extern "C" {

// One launch of the read stream over `bytes` (a multiple of 16) at device pointer d_buf.
int roof_read_stream(const void *d_buf, uint64_t bytes, int grid, int block, uint32_t *d_sink, void *stream) {
    if (!d_buf || bytes % 16 != 0 || grid < 1 || block != 256 || !d_sink) return -1;
    hipLaunchKernelGGL(read_stream_kernel, dim3(grid), dim3(block), 0, (hipStream_t)stream,
                       (const u32x4 *)d_buf, bytes / 16, 0xA5A5A5A5u, d_sink);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// One launch of `grid` workgroups of `block` threads, each lane issuing iters * 16 LDS atomic
// increments at `pattern`; d_out[grid] receives each workgroup's table total.
int roof_lds_atomics(int pattern, int iters, int grid, int block, uint32_t *d_out, void *stream) {
    if (iters < 1 || grid < 1 || block < 64 || block > 1024 || block % 64 != 0 || !d_out) return -1;
    const hipStream_t s = (hipStream_t)stream;
    const size_t lds = 33u * kRowWords * sizeof(uint32_t);
    switch (pattern) {
        case PAT_DISTINCT: hipLaunchKernelGGL(lds_atomic_kernel<PAT_DISTINCT>, dim3(grid), dim3(block), lds, s, iters, 7u, d_out, kRowWords); break;
        case PAT_RAND256: hipLaunchKernelGGL(lds_atomic_kernel<PAT_RAND256>, dim3(grid), dim3(block), lds, s, iters, 7u, d_out, kRowWords); break;
        case PAT_BAND: hipLaunchKernelGGL(lds_atomic_kernel<PAT_BAND>, dim3(grid), dim3(block), lds, s, iters, 7u, d_out, kRowWords); break;
        case PAT_SMOOTH: hipLaunchKernelGGL(lds_atomic_kernel<PAT_SMOOTH>, dim3(grid), dim3(block), lds, s, iters, 7u, d_out, kRowWords); break;
        case PAT_SAME: hipLaunchKernelGGL(lds_atomic_kernel<PAT_SAME>, dim3(grid), dim3(block), lds, s, iters, 7u, d_out, kRowWords); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// Atomic increments one roof_lds_atomics launch issues per lane (iters * this).
int roof_lds_atomics_per_iter(void) { return kUnroll; }

}  // extern "C"
