// gfx950 kernels for Köhler's contrast curve (G. Noyel, arXiv 1707.05062).
//
// What one launch computes, per image (Sec. 2.1, eqs (1)-(4)): for every integer threshold t,
// sum(t) = sum over B(t) of min(f(x1) - t, t - f(x0)), count(t) = #B(t), C(t) = sum(t) / count(t),
// the local maxima of C and the optimum t0.
//
// Route (same integers as Algorithm 1 of Sec. 3.1 over the half neighbourhood of Sec. 3.2):
//  * Each unordered neighbour pair {p, q} is visited once (half neighbourhood N4* = {right, down},
//    N8* adds {down-right, down-left}, eq (9)). With lo = min, hi = max and gap d = hi - lo, the pair
//    is in B(t) exactly for lo <= t < hi and contributes the tent min(hi - t, t - lo) to sum(t).
//  * Instead of walking t over [lo, hi) as Algorithm 1 does, every pair becomes O(1) updates of
//    difference arrays: count(t) is the prefix sum of D1 with D1[lo] += 1, D1[hi] -= 1, and sum(t)
//    is the double prefix sum of E with E[lo+1] += 1, E[floor((lo+hi)/2)+1] -= 1,
//    E[ceil((lo+hi)/2)+1] -= 1, E[hi+1] += 1. Both depend on the pair only through three
//    histograms: of lo (hmin), of hi (hmax) and of lo+hi (hsum).
//  * Those histograms are accumulated per workgroup in LDS:
//      FORM_BAND (M <= 256): a joint histogram of (d, lo) for gaps 1..band, one LDS atomic per pair;
//                 rarer larger gaps go to small hmin/hmax/hsum tables (three atomics). Gap-0 pairs
//                 add nothing to either array and are skipped. The joint table is projected onto the
//                 three marginals afterwards: rows give hmin, diagonals hmax, anti-diagonals hsum.
//      FORM_MARG  (M up to 10200): hmin and hsum per pair plus a per-pixel histogram weighted by the
//                 number of neighbours, hdeg = hmin + hmax.
//  * Each workgroup turns its histograms into D1 and E and adds them to the image's int64
//    accumulators with global atomics. The workgroup that completes an image's last unit of work
//    (a per-image counter) runs the prefix sums, the FP64 division, the local maxima and t0, and
//    clears the accumulators for the next launch.
//
// Work decomposition: an image is cut into vertical strips of 64 * K columns (K pixels per lane);
// one "unit" is one row of one strip. Units are numbered strip-major, the launch's unit space is
// split evenly over workgroups (a batch concatenates its images), and a wave walks down its rows
// keeping the row below in registers, so each pixel is read from HBM once (plus one halo row per
// wave range). Horizontal neighbours across lanes come from DPP wave shifts; only lanes 0 and 63
// load one extra pixel per row.

#include "kohler_impl.h"

namespace kohler {
namespace {

constexpr int kRing = 8;  // rows whose loads a wave keeps in flight ahead of the pair work

// Explicit address spaces keep loads, stores and atomics on the global (not flat) and LDS paths.
#define KOHLER_GLOBAL __attribute__((address_space(1)))
#define KOHLER_LDS __attribute__((address_space(3)))
typedef KOHLER_LDS uint32_t lds_u32;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ const KOHLER_GLOBAL T *gptr(const T *p) {
    return (const KOHLER_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ KOHLER_GLOBAL T *gptr(T *p) {
    return (KOHLER_GLOBAL T *)p;
}

enum : int32_t { ST_OK = 0, ST_RANGE = -2, ST_CAPACITY = -3 };

// ------------------------------------------------------------------------------------------------
// small device helpers

// DPP wave-wide shifts (GFX9 controls): lane i gets the value of lane i+1 (from_next_lane) or
// lane i-1 (from_prev_lane); the lane without a source keeps `edge`. Must run with all lanes active.
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v, uint32_t edge) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
}

__device__ __forceinline__ void lds_inc(lds_u32 *p) {
    __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(lds_u32 *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint64_t load_agent(const unsigned long long *p) {
    return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// sign(C(u) - C(v)) exactly, where C = s / k (0 when k == 0); s, k >= 0, products need 128 bits.
__device__ __forceinline__ int cmp_curve(int64_t su, int64_t ku, int64_t sv, int64_t kv) {
    const uint64_t nu = ku ? (uint64_t)su : 0, du = ku ? (uint64_t)ku : 1;
    const uint64_t nv = kv ? (uint64_t)sv : 0, dv = kv ? (uint64_t)kv : 1;
    const uint64_t lh = __umul64hi(nu, dv), ll = nu * dv;
    const uint64_t rh = __umul64hi(nv, du), rl = nv * du;
    if (lh != rh) return lh > rh ? 1 : -1;
    if (ll != rl) return ll > rl ? 1 : -1;
    return 0;
}

struct BlockScratch {
    int64_t scan[16];
    int64_t red_s[16];
    int64_t red_k[16];
    int32_t red_t[16];
    int32_t last;
};

// Inclusive prefix sum over the workgroup (blockDim.x a multiple of 64, at most 1024 threads).
__device__ int64_t block_scan(int64_t x, BlockScratch &bs, int64_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) bs.scan[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < nw; ++w) {
            run += bs.scan[w];
            bs.scan[w] = run;
        }
    }
    __syncthreads();
    if (wid > 0) x += bs.scan[wid - 1];
    total = bs.scan[nw - 1];
    __syncthreads();
    return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

// ------------------------------------------------------------------------------------------------
// pixel loading: K pixels per lane per row, packed in NW dwords

template <typename Pix, int K>
struct Packed {
    static constexpr int NW = (K * (int)sizeof(Pix)) / 4;
};

template <typename Pix, int K>
__device__ __forceinline__ void load_chunk(const Pix *row, int c, int W, bool vec,
                                           uint32_t (&w)[Packed<Pix, K>::NW]) {
    constexpr int NW = Packed<Pix, K>::NW;
    if (vec && c + K <= W) {
        if constexpr (NW == 1) {
            w[0] = *gptr(reinterpret_cast<const uint32_t *>(row + c));
        } else if constexpr (NW == 2) {
            const u32x2 t = *gptr(reinterpret_cast<const u32x2 *>(row + c));
            w[0] = t.x;
            w[1] = t.y;
        } else {
            const u32x4 t = *gptr(reinterpret_cast<const u32x4 *>(row + c));
            w[0] = t.x;
            w[1] = t.y;
            w[2] = t.z;
            w[3] = t.w;
        }
    } else {
        constexpr int PPW = 4 / (int)sizeof(Pix);
        constexpr int SH = 8 * (int)sizeof(Pix);
#pragma unroll
        for (int q = 0; q < NW; ++q) w[q] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t e = (c + k < W) ? (uint32_t)gptr(row)[c + k] : 0u;
            w[k / PPW] |= e << (SH * (k % PPW));
        }
    }
}

template <typename Pix, int K>
__device__ __forceinline__ void unpack(const uint32_t (&w)[Packed<Pix, K>::NW], uint32_t (&v)[K]) {
    constexpr int PPW = 4 / (int)sizeof(Pix);
    constexpr int SH = 8 * (int)sizeof(Pix);
    constexpr uint32_t MASK = (sizeof(Pix) == 1) ? 0xFFu : 0xFFFFu;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (w[k / PPW] >> (SH * (k % PPW))) & MASK;
}

// ------------------------------------------------------------------------------------------------
// per-pair accumulators (LDS)

// Joint histogram of (gap, low value) for gaps 1..nb, row stride 256; spill marginals for larger gaps.
struct BandAcc {
    lds_u32 *band, *smin, *smax, *ssum;
    uint32_t nb;
    __device__ __forceinline__ void pair(uint32_t x, uint32_t y, bool valid) {
        y = valid ? y : x;  // an invalid pair becomes a gap-0 pair, which contributes nothing
        const uint32_t a = min(x, y);
        const uint32_t d = max(x, y) - a;
        if (d - 1u < nb) {
            lds_inc(&band[(d - 1u) * 256u + a]);
        } else if (d > nb) {
            lds_inc(&smin[a]);
            lds_inc(&smax[a + d]);
            lds_inc(&ssum[2u * a + d]);
        }
    }
    __device__ __forceinline__ void pixel(uint32_t, uint32_t, bool) {}
    static constexpr bool kPixels = false;
};

// Marginal histograms: low value and value sum per pair, degree-weighted value per pixel.
struct MargAcc {
    lds_u32 *hmin, *hdeg, *hsum;
    __device__ __forceinline__ void pair(uint32_t x, uint32_t y, bool valid) {
        if (valid) {
            lds_inc(&hmin[min(x, y)]);
            lds_inc(&hsum[x + y]);
        }
    }
    __device__ __forceinline__ void pixel(uint32_t v, uint32_t deg, bool valid) {
        if (valid) lds_add(&hdeg[v], deg);
    }
    static constexpr bool kPixels = true;
};

// ------------------------------------------------------------------------------------------------
// pair formation for one row of one strip

// FULL: every column of the strip and the column right of it lie inside the image, so no
// per-column test is needed (all strips but the last one of a row).
template <int NB, int K, bool FULL, class Acc>
__device__ __forceinline__ void row_pairs(const uint32_t (&cur)[K], const uint32_t (&nxt)[K],
                                          uint32_t er_cur, uint32_t er_nxt, uint32_t el_nxt,
                                          bool has_up, bool has_down, int c, int W, Acc &acc) {
    // right neighbour of this lane's last pixel: next lane's first pixel, or the edge load (lane 63)
    const uint32_t rn = from_next_lane(cur[0], er_cur);
#pragma unroll
    for (int k = 0; k + 1 < K; ++k) acc.pair(cur[k], cur[k + 1], FULL || c + k + 1 < W);
    acc.pair(cur[K - 1], rn, FULL || c + K < W);
    if (has_down) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc.pair(cur[k], nxt[k], FULL || c + k < W);
        if constexpr (NB == 8) {
            const uint32_t rnd = from_next_lane(nxt[0], er_nxt);
            const uint32_t lnd = from_prev_lane(nxt[K - 1], el_nxt);
#pragma unroll
            for (int k = 0; k + 1 < K; ++k) acc.pair(cur[k], nxt[k + 1], FULL || c + k + 1 < W);
            acc.pair(cur[K - 1], rnd, FULL || c + K < W);
            acc.pair(cur[0], lnd, c >= 1 && (FULL || c < W));
#pragma unroll
            for (int k = 1; k < K; ++k) acc.pair(cur[k], nxt[k - 1], FULL || c + k < W);
        }
    }
    if constexpr (Acc::kPixels) {
        const uint32_t vert = (uint32_t)has_up + (uint32_t)has_down;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int x = c + k;
            const uint32_t horz = (uint32_t)(x > 0) + (uint32_t)(x + 1 < W);
            const uint32_t deg = (NB == 4) ? vert + horz : (vert + 1) * (horz + 1) - 1;
            acc.pixel(cur[k], deg, FULL || x < W);
        }
    }
}

// One row of packed pixels in flight: the lane's K pixels plus the edge pixels lanes 63 and 0 need.
template <int NW>
struct RowSlot {
    uint32_t w[NW];
    uint32_t er, el;
};

template <typename Pix, int NB, int K>
__device__ __forceinline__ void load_slot(const Pix *row, int c, int W, bool vec, int lane,
                                          RowSlot<Packed<Pix, K>::NW> &sl) {
    load_chunk<Pix, K>(row, c, W, vec, sl.w);
    sl.er = 0;
    sl.el = 0;
    if (lane == 63 && c + K < W) sl.er = gptr(row)[c + K];
    if (NB == 8 && lane == 0 && c >= 1) sl.el = gptr(row)[c - 1];
}

// Rows [r0, r1) of strip s, by one wave. Loads run kRing rows ahead of the pair work: the ring slot
// of a row is fixed by unrolling, so the ring stays in registers.
template <typename Pix, int NB, int K, bool CLAMP, bool FULL, class Acc>
__device__ __forceinline__ void strip_rows(const KImage &im, int s, int64_t r0, int64_t r1, uint32_t Mm1, Acc &acc,
                           uint32_t &vmax) {
    constexpr int NW = Packed<Pix, K>::NW;
    constexpr int SW = 64 * K;
    const int lane = threadIdx.x & 63;
    const Pix *base = static_cast<const Pix *>(im.ptr);
    const int64_t H = im.H, pitch = im.pitch;
    const int W = (int)im.W;
    const int c = s * SW + lane * K;
    const bool vec = im.vec_ok != 0;

    RowSlot<NW> ring[kRing];
#pragma unroll
    for (int j = 0; j < kRing; ++j) {
        const int64_t row = r0 + j;
        if (row <= r1 && row < H) load_slot<Pix, NB, K>(base + row * pitch, c, W, vec, lane, ring[j]);
    }
    for (int64_t r = r0; r < r1; r += kRing) {
#pragma unroll
        for (int j = 0; j < kRing; ++j) {
            const int64_t row = r + j;
            if (row < r1) {
                const bool has_down = row + 1 < H;
                const RowSlot<NW> &a = ring[j];
                const RowSlot<NW> &b = ring[(j + 1) % kRing];
                uint32_t cur[K], nxt[K];
                unpack<Pix, K>(a.w, cur);
                unpack<Pix, K>(b.w, nxt);
                uint32_t e0 = a.er, e1 = b.er, l1 = b.el;
                if constexpr (CLAMP) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        vmax = max(vmax, cur[k]);
                        cur[k] = min(cur[k], Mm1);
                        nxt[k] = min(nxt[k], Mm1);
                    }
                    e0 = min(e0, Mm1);
                    e1 = min(e1, Mm1);
                    l1 = min(l1, Mm1);
                }
                row_pairs<NB, K, FULL>(cur, nxt, e0, e1, l1, row > 0, has_down, c, W, acc);
                const int64_t nrow = row + kRing;
                if (nrow <= r1 && nrow < H) load_slot<Pix, NB, K>(base + nrow * pitch, c, W, vec, lane, ring[j]);
            }
        }
    }
}

// Units [la, lb) of one image (image-local, strip-major), by one wave.
template <typename Pix, int NB, int K, bool CLAMP, class Acc>
__device__ __forceinline__ void wave_units(const KImage &im, int64_t la, int64_t lb, uint32_t Mm1, Acc &acc,
                           uint32_t &vmax) {
    constexpr int SW = 64 * K;
    int64_t u = la;
    while (u < lb) {
        const int s = (int)(u / im.H);
        const int64_t r = u - (int64_t)s * im.H;
        const int64_t rend = min(im.H, r + (lb - u));
        if ((int64_t)(s + 1) * SW < im.W)
            strip_rows<Pix, NB, K, CLAMP, true>(im, s, r, rend, Mm1, acc, vmax);
        else
            strip_rows<Pix, NB, K, CLAMP, false>(im, s, r, rend, Mm1, acc, vmax);
        u += rend - r;
    }
}

// ------------------------------------------------------------------------------------------------
// histograms -> difference arrays -> global accumulators

__device__ __forceinline__ void add_global(int64_t *p, int64_t v) {
    if (v != 0)
        __hip_atomic_fetch_add(gptr(reinterpret_cast<unsigned long long *>(p)), (unsigned long long)v,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// E[v] for v >= 1 from the marginals at v-1: hmin + hmax - hsum[2v-3] - 2 hsum[2v-2] - hsum[2v-1].
__device__ __forceinline__ int64_t second_diff(int64_t lohi, const lds_u32 *hsum, int v, int M) {
    const int s = 2 * v - 2;
    int64_t e = lohi - 2 * (int64_t)hsum[s];
    if (s >= 1) e -= hsum[s - 1];
    if (s + 1 <= 2 * M - 2) e -= hsum[s + 1];
    return e;
}

__device__ __forceinline__ void merge_band(const KParams &p, lds_u32 *lds, int64_t *acc) {
    const int M = p.M;
    const uint32_t nb = (uint32_t)p.band;
    lds_u32 *band = lds, *smin = lds + nb * 256u, *smax = smin + 256, *ssum = smax + 256;
    // project the joint table on rows (hmin), diagonals (hmax) and anti-diagonals (hsum), in place
    for (int x = threadIdx.x; x < 4 * M - 1; x += blockDim.x) {
        if (x < M) {
            const int v = x;
            uint32_t r = smin[v];
            for (uint32_t d = 1; d <= nb; ++d) r += band[(d - 1) * 256u + v];
            smin[v] = r;
        } else if (x < 2 * M) {
            const int v = x - M;
            uint32_t q = smax[v];
            const uint32_t dm = min(nb, (uint32_t)v);
            for (uint32_t d = 1; d <= dm; ++d) q += band[(d - 1) * 256u + v - d];
            smax[v] = q;
        } else {
            const int s = x - 2 * M;
            uint32_t q = ssum[s];
            const uint32_t dm = min(nb, (uint32_t)s);
            for (uint32_t d = 2 - (s & 1); d <= dm; d += 2) q += band[(d - 1) * 256u + (s - d) / 2];
            ssum[s] = q;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < M; v += blockDim.x) {
        add_global(acc + v, (int64_t)smin[v] - (int64_t)smax[v]);
        if (v >= 1) add_global(acc + M + v, second_diff((int64_t)smin[v - 1] + smax[v - 1], ssum, v, M));
    }
}

__device__ __forceinline__ void merge_marg(const KParams &p, lds_u32 *lds, int64_t *acc) {
    const int M = p.M;
    const lds_u32 *hmin = lds, *hdeg = lds + M, *hsum = lds + 2 * M;
    for (int v = threadIdx.x; v < M; v += blockDim.x) {
        add_global(acc + v, 2 * (int64_t)hmin[v] - (int64_t)hdeg[v]);
        if (v >= 1) add_global(acc + M + v, second_diff((int64_t)hdeg[v - 1], hsum, v, M));
    }
}

// ------------------------------------------------------------------------------------------------
// finalize: prefix sums, C, local maxima and t0 for image i (run by one workgroup)

__device__ __forceinline__ void finalize(const KParams &p, int i, KOHLER_LDS int8_t *rel, BlockScratch &bs) {
    const int M = p.M, tid = threadIdx.x, nt = blockDim.x;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(p.acc + (int64_t)i * 2 * M);
    int64_t *osum = p.sum + (int64_t)i * M;
    int64_t *ocnt = p.count + (int64_t)i * M;
    double *oC = p.C + (int64_t)i * M;

    int64_t carK = 0, car1 = 0, car2 = 0, tot;
    for (int b = 0; b < M; b += nt) {
        const int t = b + tid;
        const bool in = t < M;
        int64_t d1 = 0, e = 0;
        if (in) {
            d1 = (int64_t)load_agent(acc + t);
            e = (int64_t)load_agent(acc + M + t);
            store_agent(acc + t, 0);
            store_agent(acc + M + t, 0);
        }
        const int64_t cnt = carK + block_scan(d1, bs, tot);
        carK += tot;
        const int64_t delta = car1 + block_scan(e, bs, tot);
        car1 += tot;
        const int64_t sm = car2 + block_scan(in ? delta : 0, bs, tot);
        car2 += tot;
        if (in) {
            osum[t] = sm;
            ocnt[t] = cnt;
            oC[t] = cnt ? (double)sm / (double)cnt : 0.0;
        }
    }
    __syncthreads();

    // rel[t] = sign(C(t) - C(t-1))
    for (int t = tid; t < M; t += nt)
        rel[t] = (int8_t)(t == 0 ? 0 : cmp_curve(osum[t], ocnt[t], osum[t - 1], ocnt[t - 1]));
    __syncthreads();

    // local maxima: a run start (t == 0 or a rise) with positive C whose run ends in a fall or at M
    int32_t *othr = p.thr + (int64_t)i * p.cap;
    int64_t found = 0;
    for (int b = 0; b < M; b += nt) {
        const int t = b + tid;
        int64_t flag = 0;
        if (t < M && (t == 0 || rel[t] > 0) && cmp_curve(osum[t], ocnt[t], 0, 1) > 0) {
            int u = t + 1;
            while (u < M && rel[u] == 0) ++u;
            flag = (u == M || rel[u] < 0) ? 1 : 0;
        }
        const int64_t pos = found + block_scan(flag, bs, tot) - flag;
        if (flag && pos < p.cap) othr[pos] = t;
        found += tot;
    }

    // t0: smallest t attaining max C
    int32_t bt = -1;
    int64_t bsum = 0, bcnt = 0;
    for (int t = tid; t < M; t += nt) {
        if (bt < 0 || cmp_curve(osum[t], ocnt[t], bsum, bcnt) > 0) {
            bt = t;
            bsum = osum[t];
            bcnt = ocnt[t];
        }
    }
    // wave reduction, then across waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int32_t ot = __shfl_down(bt, off, 64);
        const int64_t os = __shfl_down(bsum, off, 64);
        const int64_t ok = __shfl_down(bcnt, off, 64);
        if ((tid & 63) + off < 64 && ot >= 0) {
            const int c = bt < 0 ? 1 : cmp_curve(os, ok, bsum, bcnt);
            if (c > 0 || (c == 0 && ot < bt)) {
                bt = ot;
                bsum = os;
                bcnt = ok;
            }
        }
    }
    if ((tid & 63) == 0) {
        bs.red_t[tid >> 6] = bt;
        bs.red_s[tid >> 6] = bsum;
        bs.red_k[tid >> 6] = bcnt;
    }
    __syncthreads();
    if (tid == 0) {
        int32_t t0 = -1;
        int64_t s0 = 0, k0 = 0;
        for (int w = 0; w < (nt >> 6); ++w) {
            const int32_t ot = bs.red_t[w];
            if (ot < 0) continue;
            const int c = t0 < 0 ? 1 : cmp_curve(bs.red_s[w], bs.red_k[w], s0, k0);
            if (c > 0 || (c == 0 && ot < t0)) {
                t0 = ot;
                s0 = bs.red_s[w];
                k0 = bs.red_k[w];
            }
        }
        if (t0 >= 0 && cmp_curve(s0, k0, 0, 1) <= 0) t0 = -1;
        const uint32_t rf = __hip_atomic_load(gptr(p.rflag + i), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(gptr(p.rflag + i), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        store_agent(p.done + i, 0);
        p.n_thr[i] = (int32_t)found;
        p.t0[i] = t0;
        p.status[i] = rf ? ST_RANGE : (found > p.cap ? ST_CAPACITY : ST_OK);
    }
}

// ------------------------------------------------------------------------------------------------
// the kernel

__device__ __forceinline__ int find_image(const KParams &p, int64_t u) {
    int lo = 0, hi = p.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gptr(p.imgs)[mid].ustart <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The descriptor of image i, with every field wave-uniform (scalar registers).
__device__ __forceinline__ KImage image_desc(const KParams &p, int i) {
    KImage im = p.img0;
    if (p.n != 1) {
        const KOHLER_GLOBAL KImage *q = gptr(p.imgs) + i;
        im.ptr = q->ptr;
        im.H = q->H;
        im.W = q->W;
        im.pitch = q->pitch;
        im.ustart = q->ustart;
        im.nunits = q->nunits;
        im.nstrips = q->nstrips;
        im.vec_ok = q->vec_ok;
    }
    im.ptr = (const void *)uniform64((int64_t)im.ptr);
    im.H = uniform64(im.H);
    im.W = uniform64(im.W);
    im.pitch = uniform64(im.pitch);
    im.ustart = uniform64(im.ustart);
    im.nunits = uniform64(im.nunits);
    im.nstrips = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)im.nstrips);
    im.vec_ok = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)im.vec_ok);
    return im;
}

template <typename Pix, int NB, int K, int FORM, bool CLAMP>
__global__ void __launch_bounds__(512) curve_kernel(KParams p) {
    extern __shared__ __align__(16) uint32_t lds_raw[];
    __shared__ BlockScratch bs;
    lds_u32 *lds = (lds_u32 *)lds_raw;

    const int G = gridDim.x;
    // consecutive logical workgroups land on the same XCD (the dispatcher deals blocks round-robin)
    const int g = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const int64_t U = p.total_units;
    int64_t u = (int64_t)g * U / G;
    const int64_t uend = (int64_t)(g + 1) * U / G;
    const int nw = blockDim.x >> 6, wid = threadIdx.x >> 6;
    const uint32_t Mm1 = (uint32_t)p.M - 1u;

    uint32_t table_words;
    if constexpr (FORM == FORM_BAND) table_words = (uint32_t)p.band * 256u + 1024u;
    else table_words = 4u * (uint32_t)p.M;

    while (u < uend) {
        const int i = (p.n == 1) ? 0 : find_image(p, u);
        const KImage im = image_desc(p, i);
        const int64_t seg_end = min(uend, im.ustart + im.nunits);
        const int64_t nseg = seg_end - u;

        for (uint32_t x = threadIdx.x; x < table_words / 4; x += blockDim.x)
            reinterpret_cast<KOHLER_LDS u32x4 *>(lds)[x] = u32x4{0u, 0u, 0u, 0u};
        __syncthreads();

        const int64_t lbase = u - im.ustart;
        const int64_t la = lbase + wid * nseg / nw, lb = lbase + (wid + 1) * nseg / nw;
        uint32_t vmax = 0;
        if constexpr (FORM == FORM_BAND) {
            const uint32_t nb = (uint32_t)p.band;
            BandAcc acc{lds, lds + nb * 256u, lds + nb * 256u + 256u, lds + nb * 256u + 512u, nb};
            wave_units<Pix, NB, K, CLAMP>(im, la, lb, Mm1, acc, vmax);
        } else {
            MargAcc acc{lds, lds + p.M, lds + 2 * p.M};
            wave_units<Pix, NB, K, CLAMP>(im, la, lb, Mm1, acc, vmax);
        }
        if constexpr (CLAMP) {
            vmax = wave_max(vmax);
            if ((threadIdx.x & 63) == 0 && vmax > Mm1)
                __hip_atomic_fetch_or(gptr(p.rflag + i), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();

        int64_t *acc_g = p.acc + (int64_t)i * 2 * p.M;
        if constexpr (FORM == FORM_BAND) merge_band(p, lds, acc_g);
        else merge_marg(p, lds, acc_g);

        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long old = __hip_atomic_fetch_add(
                gptr(p.done + i), (unsigned long long)nseg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bs.last = (old + (unsigned long long)nseg == (unsigned long long)im.nunits) ? 1 : 0;
        }
        __syncthreads();
        if (bs.last) {
            __threadfence();
            finalize(p, i, (KOHLER_LDS int8_t *)lds, bs);
        }
        __syncthreads();
        u = seg_end;
    }
}

template <typename Pix, int NB, int K>
const void *pick_form(int form, bool clamp) {
    if (form == FORM_BAND)
        return clamp ? reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_BAND, true>)
                     : reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_BAND, false>);
    return clamp ? reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_MARG, true>)
                 : reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_MARG, false>);
}

// The kernel instance for a launch family; pixel values are clamped (and range-checked) unless the
// dtype cannot exceed M - 1 (uint8 with M = 256).
const void *pick_kernel(int dtype, int nbhd, int form, int px_per_lane, int M) {
    if (dtype == 1) {
        const bool clamp = M < 256;
        if (nbhd == 4) return px_per_lane == 8 ? pick_form<uint8_t, 4, 8>(form, clamp) : pick_form<uint8_t, 4, 4>(form, clamp);
        return px_per_lane == 8 ? pick_form<uint8_t, 8, 8>(form, clamp) : pick_form<uint8_t, 8, 4>(form, clamp);
    }
    return nbhd == 4 ? pick_form<uint16_t, 4, 4>(form, true) : pick_form<uint16_t, 8, 4>(form, true);
}

hipError_t allow_large_lds(const void *kern) {
    return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(kMaxLdsBytes - sizeof(BlockScratch) - 64));
}

}  // namespace

size_t lds_bytes(int form, int M, int band) {
    size_t words = (form == FORM_BAND) ? (size_t)band * 256 + 1024 : 4 * (size_t)M;
    size_t bytes = words * 4;
    const size_t need_fin = ((size_t)M + 15) & ~(size_t)15;  // rel[] of the finalize step
    return bytes > need_fin ? bytes : need_fin;
}

hipError_t launch_curve(const KParams &p, int dtype, int nbhd, int form, int px_per_lane, int block,
                        int grid, hipStream_t stream) {
    const size_t lds = lds_bytes(form, p.M, p.band);
    const void *kern = pick_kernel(dtype, nbhd, form, px_per_lane, p.M);
    hipError_t e = allow_large_lds(kern);
    if (e != hipSuccess) return e;
    KParams arg = p;
    void *args[] = {&arg};
    e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

int blocks_per_cu(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block) {
    const void *kern = pick_kernel(dtype, nbhd, form, px_per_lane, M);
    if (allow_large_lds(kern) != hipSuccess) return 1;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block, lds_bytes(form, M, band)) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

}  // namespace kohler
