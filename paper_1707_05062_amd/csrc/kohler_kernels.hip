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

#include <mutex>
#include <type_traits>

#include "kohler_impl.h"
#include "kohler_columns.h"

namespace kohler {
namespace {


// Explicit address spaces keep loads, stores and atomics on the global (not flat) and LDS paths.
#define KOHLER_GLOBAL __attribute__((address_space(1)))
#define KOHLER_LDS __attribute__((address_space(3)))
typedef KOHLER_LDS uint32_t lds_u32;

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));  // two 16-bit lanes of one VGPR (v_pk_* ops)

__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

template <typename T>
__device__ __forceinline__ const KOHLER_GLOBAL T *gptr(const T *p) {
    return (const KOHLER_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ KOHLER_GLOBAL T *gptr(T *p) {
    return (KOHLER_GLOBAL T *)p;
}

enum : int32_t { ST_OK = 0, ST_RANGE = -2, ST_CAPACITY = -3, ST_LAYOUT = -5 };

// Measurement build only (-DKOHLER_PHASE_CLOCK): each workgroup of the curve kernel records the
// constant 100 MHz real-time counter at its phase boundaries, and each wave the end of its pair
// work, in device arrays that kohler_phase_clock_read copies out. Slots per workgroup:
//   0 entry, 1 tables cleared, 2 every wave's pairs done, 3 projection on the marginals done,
//   4 merge atomics performed, 5 ticket taken, 6 finishing workgroup: replicas gathered,
//   7 finishing workgroup: done, 8 the hardware id register of the workgroup's first wave (compute
//   unit, shader array, engine), 9 the id of its accelerator complex die (XCD), 10 and 11 the
//   shader clock (cycles) at stamps 6 and 7, 12 .. 14 the shader clock at the finishing
//   workgroup's three barriers (clock_stamp).
#ifdef KOHLER_PHASE_CLOCK
constexpr int kPhaseSlots = 16;
constexpr int kPhaseMaxWG = 4096;
constexpr int kPhaseWaves = 16;
__device__ unsigned long long g_phase[kPhaseMaxWG * kPhaseSlots];
__device__ unsigned long long g_phase_wave[kPhaseMaxWG * kPhaseWaves];
__device__ __forceinline__ void phase_stamp(int slot) {
    if (threadIdx.x == 0 && blockIdx.x < (unsigned)kPhaseMaxWG) {
        gptr(g_phase)[blockIdx.x * kPhaseSlots + slot] = (unsigned long long)wall_clock64();
        if (slot == 6 || slot == 7) gptr(g_phase)[blockIdx.x * kPhaseSlots + slot + 4] = (unsigned long long)clock64();
    }
}
__device__ __forceinline__ void clock_stamp(int slot) {
    if (threadIdx.x == 0 && blockIdx.x < (unsigned)kPhaseMaxWG)
        gptr(g_phase)[blockIdx.x * kPhaseSlots + slot] = (unsigned long long)clock64();
}
__device__ __forceinline__ void phase_place() {
    if (threadIdx.x == 0 && blockIdx.x < (unsigned)kPhaseMaxWG) {
        gptr(g_phase)[blockIdx.x * kPhaseSlots + 8] = __builtin_amdgcn_s_getreg(4 | (31 << 11));
        gptr(g_phase)[blockIdx.x * kPhaseSlots + 9] = __builtin_amdgcn_s_getreg(20 | (15 << 11));
    }
}
__device__ __forceinline__ void phase_wave_stamp() {
    const unsigned w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0 && blockIdx.x < (unsigned)kPhaseMaxWG && w < (unsigned)kPhaseWaves)
        gptr(g_phase_wave)[blockIdx.x * kPhaseWaves + w] = (unsigned long long)wall_clock64();
}
#else
__device__ __forceinline__ void phase_stamp(int) {}
__device__ __forceinline__ void clock_stamp(int) {}
__device__ __forceinline__ void phase_place() {}
__device__ __forceinline__ void phase_wave_stamp() {}
#endif

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

// LDS word at a byte address counted from the start of the workgroup's LDS. The kernel declares no
// static LDS, so its dynamic LDS (the histogram table first) starts at address 0; the kernel checks
// this at entry.
__device__ __forceinline__ lds_u32 *lds_at(uint32_t byte_addr) { return (lds_u32 *)(size_t)byte_addr; }

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it does not wait for the
// wave's global loads, which stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void lds_inc(lds_u32 *p) {
    __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(lds_u32 *p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Data shared between workgroups (image accumulators, unit counters, range flags) is only touched
// with system-scope atomics, which are performed past the per-XCD L2 caches. That keeps every
// workgroup's view coherent without agent-scope fences, which on this chip write back and
// invalidate the whole L2. A workgroup makes its contributions visible before it takes its ticket
// by using returning atomics and waiting for their results.
#define KOHLER_XSCOPE __HIP_MEMORY_SCOPE_SYSTEM

__device__ __forceinline__ uint64_t load_shared(const unsigned long long *p) {
    return __hip_atomic_load(gptr(p), __ATOMIC_RELAXED, KOHLER_XSCOPE);
}
__device__ __forceinline__ void store_shared(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(gptr(p), v, __ATOMIC_RELAXED, KOHLER_XSCOPE);
}
__device__ __forceinline__ uint64_t add_shared(unsigned long long *p, unsigned long long v) {
    return __hip_atomic_fetch_add(gptr(p), v, __ATOMIC_RELAXED, KOHLER_XSCOPE);
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

typedef KOHLER_LDS BlockScratch LdsScratch;


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

// K pixels of one row. Every lane issues its loads unconditionally: a load whose destination
// another lane's path overwrites while it is in flight, or whose value is used at once, makes the
// compiler drain every outstanding load, which would serialise the row ring below.
//   PACKED: one vector load of K pixels (full strips with aligned rows); unpacked when used.
//   else:   K element loads from clamped, always valid columns; the values beyond the image are
//           zeroed when used (ragged last strips, misaligned rows).
// The strip's edge columns (the pixel right of the strip, and left of it for 8 neighbours) are not
// part of a slot: a batch loads them for all its rows at once (strip_rows).
template <typename Pix, int K, bool PACKED>
struct RowSlot {
    static constexpr int NV = PACKED ? Packed<Pix, K>::NW : K;
    uint32_t v[NV];
};

template <typename Pix, int K, bool FULL, bool PACKED>
__device__ __forceinline__ void load_slot(const Pix *row, int c, int W, RowSlot<Pix, K, PACKED> &sl) {
    constexpr int NW = Packed<Pix, K>::NW;
    // column offsets are unsigned 32-bit, so each load is a wave-uniform row address (scalar
    // registers) plus a zero-extended per-lane offset
    const KOHLER_GLOBAL Pix *rp = gptr(row);
    if constexpr (PACKED) {
        // the last strip of a row is packed only when W is a multiple of K: lanes past the row
        // end re-read the row's last aligned chunk, and their pairs are masked out
        const uint32_t cv = (uint32_t)packed_column(c, K, W, FULL);
        if constexpr (NW == 1) {
            sl.v[0] = *reinterpret_cast<const KOHLER_GLOBAL uint32_t *>(rp + cv);
        } else if constexpr (NW == 2) {
            const u32x2 t = *reinterpret_cast<const KOHLER_GLOBAL u32x2 *>(rp + cv);
            sl.v[0] = t.x;
            sl.v[1] = t.y;
        } else {
            const u32x4 t = *reinterpret_cast<const KOHLER_GLOBAL u32x4 *>(rp + cv);
            sl.v[0] = t.x;
            sl.v[1] = t.y;
            sl.v[2] = t.z;
            sl.v[3] = t.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) sl.v[k] = (uint32_t)rp[(uint32_t)element_column(c, k, W, FULL)];
    }
}

// Pixel values of a slot, multiplied by SCALE (a power of two). Values past the row end are
// whatever was re-read (packed) or 0 (element loads); every pair that uses them is masked.
template <typename Pix, int K, bool FULL, bool PACKED, uint32_t SCALE>
__device__ __forceinline__ void slot_pixels(const RowSlot<Pix, K, PACKED> &sl, int c, int W, uint32_t (&px)[K]) {
    constexpr int SSH = SCALE == 4 ? 2 : 0;
    if constexpr (PACKED) {
        constexpr int PPW = 4 / (int)sizeof(Pix);
        constexpr int SH = 8 * (int)sizeof(Pix);
        constexpr uint32_t MASK = (sizeof(Pix) == 1) ? 0xFFu : 0xFFFFu;
#pragma unroll
        for (int k = 0; k < K; ++k) px[k] = ((sl.v[k / PPW] >> (SH * (k % PPW))) & MASK) << SSH;
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) px[k] = ((FULL || c + k < W) ? sl.v[k] : 0u) << SSH;
    }
}

// ------------------------------------------------------------------------------------------------
// per-pair accumulators (LDS)

// Joint histogram of (gap d, low value lo), rows kRowStride words apart, one LDS atomic per pair.
// The workgroup keeps `copies` (C) such tables interleaved word by word: cell (d, lo) of copy c is word
// (d * kRowStride + lo) * C + c, and lane l adds to copy l % C, so that fewer lanes of one LDS
// instruction land on the same counter (same-word atomics of one instruction are serialised) and the
// lanes of a copy spread over the banks. Rows (of every copy):
//   row 0        gap-0 pairs (at their value) and invalid pairs outside the image (at their
//                lane's column); never read back
//   rows 1..nb   the joint counts of (d, lo)
//   row nb+1     lo of the pairs with d > nb (their share of hmin)
// Pixel values arrive multiplied by 4 (kScale); with lo4 = 4*lo and d4 = 4*d a pair costs min, sad,
// min and two multiply-adds: the cell's byte address 4 (d S + lo) = min(d4, 4 (nb+1)) S + lo4, times
// C plus 4c (the table starts at LDS address 0).
// Pairs with d > nb still owe hmax and hsum; dmax tracks the lane's largest gap so that a
// wave-uniform test after each row can run SpillAcc over that row only when some lane needs it.
struct BandAcc {
    uint32_t cap4;  // 4 * (nb + 1): the large-gap row
    uint32_t nc;    // C, copies of the table
    uint32_t off4;  // 4 * this lane's copy
    uint32_t dmax;  // largest 4*d seen since the last test
    // Packed form (band_row_pairs): pixel values sit in 16-bit halves as C x + c, so that min gives
    // C lo + c and max - min gives C d.
    u16x2 mul2;     // [C, C]
    u16x2 coff;     // [c, c]
    u16x2 nfix;     // [0, c - c'] (mod 2^16): re-bases a value taken from the next lane (copy c')
    u16x2 cap2;     // [C (nb + 1), C (nb + 1)]
    u16x2 dmax2;    // bitwise OR of the C d seen since the last test, per half (see needs_spill2)
    static constexpr uint32_t kScale = 4;
    __device__ __forceinline__ void pair(uint32_t x4, uint32_t y4, bool valid) {
        if (!valid) {
            // a pair outside the image lands in row 0 at a word of its own lane: many lanes adding
            // to one shared word in the same instruction would be serialised
            x4 = y4 = 4u * (threadIdx.x & 63u);
        }
        const uint32_t lo4 = min(x4, y4);
        const uint32_t d4 = __builtin_amdgcn_sad_u16(x4, y4, 0u);  // |x4 - y4| (both below 2^16)
        dmax = max(dmax, d4);
        const uint32_t cell4 = __umul24(min(d4, cap4), (uint32_t)kRowStride) + lo4;
        lds_inc(lds_at(__umul24(cell4, nc) + off4));
    }
    __device__ __forceinline__ bool needs_spill() const { return dmax >= cap4; }
    // Two pairs at once: (x.lo, y.lo) and (x.hi, y.hi), values as C x + c (see mul2); the counter of a
    // pair is word min(C d, C (nb + 1)) * kRowStride + C lo + c, formed in the 16-bit halves (every
    // word of the tables lies below 2^16) and shifted to a byte address per half.
    __device__ __forceinline__ void pairs2(u16x2 x, u16x2 y) {
        const u16x2 lo = __builtin_elementwise_min(x, y);
        const u16x2 d = __builtin_elementwise_max(x, y) - lo;
        dmax2 = as_u16x2(as_u32(dmax2) | as_u32(d));
        const u16x2 w = __builtin_elementwise_min(d, cap2) * (uint16_t)kRowStride + lo;
        // each half times 4 is one shift with a 16-bit source selection (SDWA)
        lds_inc(lds_at((uint32_t)w.x * 4u));
        lds_inc(lds_at((uint32_t)w.y * 4u));
    }
    __device__ __forceinline__ bool needs_spill2() const {
        // the OR of the gaps is at least their maximum, so no large gap is missed; when cap2 is a
        // power of two (band + 1 = 2^k / C) the test is exact, else a row may be re-run needlessly
        return ((uint32_t)dmax2.x | (uint32_t)dmax2.y) >= (uint32_t)cap2.x;
    }
    __device__ __forceinline__ void pixel(uint32_t, uint32_t, bool) {}
    static constexpr bool kPixels = false;
    static constexpr bool kSpill = true;
    typedef uint32_t P;
    __device__ static __forceinline__ P prep(uint32_t v) { return v; }
};

// The 8 pixels of one lane's row (two packed words of bytes) as four 16-bit pairs, each half
// mapped to C x + c: a0 = [b0, b2], b0 = [b1, b3], a1 = [b4, b6], b1 = [b5, b7].
struct RowPk {
    u16x2 a0, b0, a1, b1;
};

// v_perm_b32 selectors (byte k of the result = source byte s_k; 0x0c gives zero; the second operand
// is bytes 0..3, the first 4..7).
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
constexpr uint32_t kSelEven = 0x0c020c00u;  // [byte 0, byte 2] as two 16-bit halves
constexpr uint32_t kSelOdd = 0x0c030c01u;   // [byte 1, byte 3]
constexpr uint32_t kSelHiLo = 0x05040302u;  // [high half of the second operand, low half of the first]

__device__ __forceinline__ RowPk row_pk(uint32_t w0, uint32_t w1, u16x2 mul, u16x2 coff) {
    RowPk r;
    r.a0 = as_u16x2(perm(0u, w0, kSelEven)) * mul + coff;
    r.b0 = as_u16x2(perm(0u, w0, kSelOdd)) * mul + coff;
    r.a1 = as_u16x2(perm(0u, w1, kSelEven)) * mul + coff;
    r.b1 = as_u16x2(perm(0u, w1, kSelOdd)) * mul + coff;
    return r;
}

// The 16 pairs of one lane's row of a full 8-bit strip in the banded form, two per call of f:
// horizontal (b0,b1)(b2,b3) | (b4,b5)(b6,b7) | (b1,b2)(b3,b4) | (b5,b6)(b7,b8), with b8 the next
// lane's b0 (lane 63: `edge`, the edge pixel times C, as copy 0 maps it), and when there is a row
// below, vertical (bk, bk') for k = 0..7. Both values of a pair carry this lane's copy offset.
template <class F>
__device__ __forceinline__ void band_row_pairs(const RowPk &r, const RowPk &n, uint32_t edge, bool has_down,
                                               u16x2 nfix, F &&f) {
    f(r.a0, r.b0);
    f(r.a1, r.b1);
    const u16x2 c0 = as_u16x2(perm(as_u32(r.a1), as_u32(r.a0), kSelHiLo));  // [b2, b4]
    f(r.b0, c0);
    // [b6, b8]: b8 from the next lane (its copy's rebasing, corrected by nfix)
    const uint32_t na0 = from_next_lane(as_u32(r.a0), edge);
    const u16x2 c1 = as_u16x2(perm(na0, as_u32(r.a1), kSelHiLo)) + nfix;
    f(r.b1, c1);
    if (has_down) {
        f(r.a0, n.a0);
        f(r.b0, n.b0);
        f(r.a1, n.a1);
        f(r.b1, n.b1);
    }
}

// Triangular joint histogram of (hi, lo) with lo <= hi, for M <= 256: one LDS atomic per pair and no
// large-gap path. Row hi starts at word T(hi) = hi (hi + 1) / 2, so the counter of a pair sits at
// byte 4 T(hi) + 4 lo = 2 (hi^2 + hi) + 4 lo. Each pixel value u is prepared once as a = 4u and
// x = u^2 + u; as x grows with u, a pair costs min(a), max(x) and one shift-add. Gap-0 pairs land
// on the diagonal, which the projection skips; pairs outside the image land on a word of their
// lane just past the table.
struct TriPx {
    uint32_t a, x;
};
struct TriAcc {
    uint32_t dummy_x;  // 2 * dummy_x is the byte address of the invalid-pair words
    uint32_t dmax, nb; // unused by this form
    static constexpr uint32_t kScale = 1;
    static constexpr bool kPixels = false;
    static constexpr bool kSpill = false;
    typedef TriPx P;
    __device__ static __forceinline__ P prep(uint32_t u) { return TriPx{u << 2, __umul24(u, u) + u}; }
    __device__ __forceinline__ void pair(P p, P q, bool valid) {
        if (!valid) {
            p.a = q.a = 4u * (threadIdx.x & 63u);
            p.x = q.x = dummy_x;
        }
        const uint32_t lo4 = min(p.a, q.a);
        const uint32_t hx = max(p.x, q.x);
        lds_inc(lds_at((hx << 1) + lo4));
    }
    __device__ __forceinline__ bool needs_spill() const { return false; }
    __device__ __forceinline__ void pixel(P, uint32_t, bool) {}
};

// Words of the triangular table for M levels (without the invalid-pair words).
__host__ __device__ constexpr uint32_t tri_words(uint32_t M) { return M * (M + 1u) / 2u; }

// Lane shifts of a prepared pixel (see from_next_lane / from_prev_lane).
__device__ __forceinline__ uint32_t next_px(uint32_t v, uint32_t edge) { return from_next_lane(v, edge); }
__device__ __forceinline__ uint32_t prev_px(uint32_t v, uint32_t edge) { return from_prev_lane(v, edge); }
__device__ __forceinline__ TriPx next_px(TriPx v, TriPx edge) {
    return TriPx{from_next_lane(v.a, edge.a), from_next_lane(v.x, edge.x)};
}
__device__ __forceinline__ TriPx prev_px(TriPx v, TriPx edge) {
    return TriPx{from_prev_lane(v.a, edge.a), from_prev_lane(v.x, edge.x)};
}

// hmax and hsum of the pairs with gap > nb (second pass over a row whose wave saw one); values
// scaled by 4, so 4*hi and 4*(lo + hi) = x4 + y4 are already byte offsets. A pair costs the gap and
// one compare unless it is one of the rare large gaps.
struct SpillAcc {
    uint32_t smax, ssum;  // byte addresses of the hmax and hsum spill tables
    uint32_t nb;
    __device__ __forceinline__ void pair(uint32_t x4, uint32_t y4, bool valid) {
        const uint32_t d4 = __builtin_amdgcn_sad_u16(x4, y4, 0u);
        if (valid && d4 > 4u * nb) {
            lds_inc(lds_at(smax + max(x4, y4)));
            lds_inc(lds_at(ssum + x4 + y4));
        }
    }
    __device__ __forceinline__ void pixel(uint32_t, uint32_t, bool) {}
    static constexpr bool kPixels = false;
    typedef uint32_t P;
};

// Marginal histograms: low value and value sum per pair, degree-weighted value per pixel.
struct MargAcc {
    // this lane's copy of each table (copy c of entry j at word j * copies + c)
    lds_u32 *hmin, *hdeg, *hsum;
    __device__ __forceinline__ void pair(uint32_t x, uint32_t y, bool valid) {
        if (valid) {
            lds_inc(hmin + (min(x, y) << cs));
            lds_inc(hsum + ((x + y) << cs));
        }
    }
    __device__ __forceinline__ void pixel(uint32_t v, uint32_t deg, bool valid) {
        if (valid) lds_add(hdeg + (v << cs), deg);
    }
    static constexpr bool kPixels = true;
    static constexpr bool kSpill = false;
    static constexpr uint32_t kScale = 1;
    uint32_t dmax, nb;
    uint32_t cs = 0;  // log2 of the table copies
    __device__ __forceinline__ bool needs_spill() const { return false; }
    typedef uint32_t P;
    __device__ static __forceinline__ P prep(uint32_t v) { return v; }
};

// ------------------------------------------------------------------------------------------------
// pair formation for one row of one strip

// FULL: every column of the strip and the column right of it lie inside the image, so no
// per-column test is needed (all strips but the last one of a row).
template <int NB, int K, bool FULL, class Acc, class P>
__device__ __forceinline__ void row_pairs(const P (&cur)[K], const P (&nxt)[K], P er_cur, P er_nxt, P el_nxt,
                                          bool has_up, bool has_down, int c, int W, Acc &acc) {
    // right neighbour of this lane's last pixel: next lane's first pixel, or the edge load (lane 63)
    const P rn = next_px(cur[0], er_cur);
#pragma unroll
    for (int k = 0; k + 1 < K; ++k) acc.pair(cur[k], cur[k + 1], FULL || c + k + 1 < W);
    acc.pair(cur[K - 1], rn, FULL || c + K < W);
    if (has_down) {
#pragma unroll
        for (int k = 0; k < K; ++k) acc.pair(cur[k], nxt[k], FULL || c + k < W);
        if constexpr (NB == 8) {
            const P rnd = next_px(nxt[0], er_nxt);
            const P lnd = prev_px(nxt[K - 1], el_nxt);
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

// Rows a wave loads together before it uses any of them (and the halo row below), chosen so that the
// kernel stays within 128 VGPRs (four waves per SIMD) without spilling: 16 rows when a lane's pixels
// of a row fit one word, else 6 (each row of a batch also costs the compiler's unpacked copies), and
// fewer where clamping or the 8-neighbourhood keep more values live. The edge pixels of all of them
// take one VGPR per side (lane j holds row j's), so at most 63 rows.
template <typename Pix, int NB, int K, bool CLAMP>
constexpr int row_batch() {
    return (K * (int)sizeof(Pix)) / 4 <= 1 ? ((CLAMP || NB == 8) ? 12 : 16) : ((CLAMP || NB == 8) ? 4 : 6);
}

// Rows of one batch of strip_rows: row_batch(), but 3 where a slot holds 8 unpacked pixels (element
// loads: ragged last strips and misaligned rows), whose ring of 8-word slots would not fit otherwise.
template <typename Pix, int NB, int K, bool CLAMP, bool PACKED>
constexpr int slot_batch() {
    return (!PACKED && K >= 8) ? 3 : row_batch<Pix, NB, K, CLAMP>();
}

// ------------------------------------------------------------------------------------------------
// Full, aligned strips of 8-bit pixels (8 per lane, 4-neighbourhood, banded form, no clamping):
// batches of kPkRows rows (longer ranges keep the next batch's loads in flight while one is used),
// with the pairs formed two per instruction (band_row_pairs). The single-image launch deals chunks
// of one batch: 4 rows balanced the waves best on the 18 MP image (3, 5, 6, 9 and 12 were slower:
// larger chunks leave the waves of a workgroup further apart, 3 rows cost more in halo loads).

#ifndef KOHLER_PK_ROWS
#define KOHLER_PK_ROWS 4
#endif
constexpr int kPkRows = KOHLER_PK_ROWS;

// The single-image launch splits each workgroup's last blockDim >> kTailShift chunks in halves.
#ifndef KOHLER_TAIL_SHIFT
#define KOHLER_TAIL_SHIFT 7
#endif
constexpr int kTailShift = KOHLER_TAIL_SHIFT;
static_assert(kPkRows >= 3 && kPkRows < 64,
              "chunks of at least 3 rows of 512 columns (chunk numbers stay 32-bit); one lane per row holds its edge pixel");

// Whether an instance takes this path (for the strips that lie wholly inside the image).
template <typename Pix, int NB, int K, bool CLAMP, class Acc>
constexpr bool pk_form() {
    return std::is_same<Acc, BandAcc>::value && std::is_same<Pix, uint8_t>::value && K == 8 && NB == 4 && !CLAMP;
}

struct PkBatch {
    RowSlot<uint8_t, 8, true> ring[kPkRows + 1];  // the rows and the halo row below
    uint32_t erv;                                 // lane j: right edge pixel of row j
    int64_t rb;                                   // first row
    int s, nr;                                    // strip, rows in the batch
};

// Issues the loads of rows [rb, r1) (r1 - rb <= kPkRows) of strip s, which lies wholly inside the
// image, and of the halo row below. The pixel right of the strip is read at column min((s + 1) 512,
// W - 1): at the image's right border that is the row's last pixel, which pairs with itself (gap 0,
// a pair that adds nothing).
__device__ __forceinline__ void pk_load(const KImage &im, int s, int64_t rb, int64_t r1, PkBatch &b) {
    constexpr int SW = 64 * 8;
    const int lane = threadIdx.x & 63;
    const uint8_t *base = static_cast<const uint8_t *>(im.ptr);
    const int64_t pitch = im.pitch;
    const int c = s * SW + lane * 8;
    const int room = (int)(min(r1, im.H - 1) - rb);  // rows past the range re-read the last one
    b.rb = rb;
    b.s = s;
    b.nr = (int)(r1 - rb);
    b.erv = (uint32_t)gptr(base + (rb + min(lane, room)) * pitch)[(uint32_t)right_edge_column(s, SW, im.W)];
    const uint8_t *rowp = base + rb * pitch;
#pragma unroll
    for (int j = 0; j <= kPkRows; ++j) {
        load_slot<uint8_t, 8, true, true>(rowp, c, (int)im.W, b.ring[j]);
        if (j < room) rowp += pitch;
    }
}

// The pairs of a loaded batch. A row with a pair of gap > nb runs the pairs again for the large-gap
// tables: with values v stored as C v + c (C a power of two <= 4), a pair (x, y) of such values has
// gap |x - y| / C, and the byte offsets of 4 max(v) and 4 (v + v') are (max(x, y) - c) << sh and
// (x + y - 2c) << sh with sh = 2 - log2 C.
template <class Spill>
__device__ __forceinline__ void pk_use(const KImage &im, const PkBatch &b, BandAcc &acc, Spill &spill) {
    const int down = (int)min<int64_t>(kPkRows, im.H - 1 - b.rb);
    const uint32_t c = acc.coff.x, c2 = 2u * c;
    const uint32_t sh = acc.nc == 1u ? 2u : (acc.nc == 2u ? 1u : 0u);
    const uint32_t cnb = acc.nc * spill.nb;
    RowPk pc = row_pk(b.ring[0].v[0], b.ring[0].v[1], acc.mul2, acc.coff);
#pragma unroll
    for (int j = 0; j < kPkRows; ++j) {
        if (j < b.nr) {
            const RowPk pn = row_pk(b.ring[j + 1].v[0], b.ring[j + 1].v[1], acc.mul2, acc.coff);
            const uint32_t edge = (uint32_t)__builtin_amdgcn_readlane((int)b.erv, j) * acc.nc;
            const bool has_down = j < down;
            band_row_pairs(pc, pn, edge, has_down, acc.nfix, [&](u16x2 x, u16x2 y) { acc.pairs2(x, y); });
            if (__any(acc.needs_spill2())) {
                band_row_pairs(pc, pn, edge, has_down, acc.nfix, [&](u16x2 x, u16x2 y) {
                    const u16x2 hi = __builtin_elementwise_max(x, y), d = hi - __builtin_elementwise_min(x, y);
                    const u16x2 t = x + y;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        if ((uint32_t)d[h] > cnb) {
                            lds_inc(lds_at(spill.smax + (((uint32_t)hi[h] - c) << sh)));
                            lds_inc(lds_at(spill.ssum + (((uint32_t)t[h] - c2) << sh)));
                        }
                    }
                });
            }
            acc.dmax2 = u16x2{0, 0};
            pc = pn;
        }
    }
}

// Rows [r0, r1) of full strip s, two batches in flight.
template <class Spill>
__device__ __forceinline__ void pk_rows(const KImage &im, int s, int64_t r0, int64_t r1, BandAcc &acc,
                                        Spill &spill) {
    PkBatch ba, bb;
    int64_t r = min(r0 + kPkRows, r1);
    pk_load(im, s, r0, r, ba);
    for (;;) {
        const bool vb = r < r1;
        if (vb) {
            const int64_t e = min(r + kPkRows, r1);
            pk_load(im, s, r, e, bb);
            r = e;
        }
        pk_use(im, ba, acc, spill);
        if (!vb) break;
        const bool va = r < r1;
        if (va) {
            const int64_t e = min(r + kPkRows, r1);
            pk_load(im, s, r, e, ba);
            r = e;
        }
        pk_use(im, bb, acc, spill);
        if (!va) break;
    }
}

// Rows [r0, r1) of strip s, by one wave, in batches of slot_batch() rows: a batch issues the loads of
// its rows and of the halo row below before it uses any of them, and uses them in order, so the
// whole batch is in flight at once and the wait before each row only covers that row.
template <typename Pix, int NB, int K, bool CLAMP, bool FULL, bool PACKED, class Acc, class Spill>
__device__ __forceinline__ void strip_rows(const KImage &im, int s, int64_t r0, int64_t r1, uint32_t Mm1,
                                           Acc &acc, Spill &spill, uint32_t &vmax) {
    constexpr int SW = 64 * K;
    constexpr int B = slot_batch<Pix, NB, K, CLAMP, PACKED>();
    const int lane = threadIdx.x & 63;
    const Pix *base = static_cast<const Pix *>(im.ptr);
    const int64_t H = im.H, pitch = im.pitch;
    const int W = (int)im.W;
    const int c = s * SW + lane * K;

    // the strip's edge columns, clamped into the image (a clamped value is never used: the pairs it
    // would form lie outside the image and are masked)
    const uint32_t cr = (uint32_t)right_edge_column(s, SW, W);
    const uint32_t cl = (uint32_t)left_edge_column(s, SW);
    static_assert(B + 1 <= 64, "one lane per row of a batch holds its edge pixels");

    // last row a batch may touch: the halo row below the range, or the image's last row
    const int64_t rlast = min(r1, H - 1);
    for (int64_t rb = r0; rb < r1; rb += B) {
        const int nr = (int)min<int64_t>(B, r1 - rb);
        RowSlot<Pix, K, PACKED> ring[B + 1];
        uint32_t erv, elv = 0;
        // unconditional loads (rows past the range re-read rlast, a cache hit): with a fixed number
        // of loads in flight the compiler can wait for exactly the row it is about to use
        {
            const int room = (int)(rlast - rb);
            // edge pixels: lane j reads those of row rb + min(j, room)
            const KOHLER_GLOBAL Pix *ep = gptr(base + (rb + min(lane, room)) * pitch);
            erv = (uint32_t)ep[cr];
            if constexpr (NB == 8) elv = (uint32_t)ep[cl];
            // row addresses by scalar increments (the rows past rlast re-read rlast)
            const Pix *rowp = base + rb * pitch;
#pragma unroll
            for (int j = 0; j <= B; ++j) {
                load_slot<Pix, K, FULL, PACKED>(rowp, c, W, ring[j]);
                if (j < room) rowp += pitch;
            }
        }
        // row rb + j has a row below when j < down, one above when j > 0 or rb > 0 (wave-uniform)
        const int down = (int)min<int64_t>(B, H - 1 - rb);
        const bool top = rb == 0;
#pragma unroll
        for (int j = 0; j < B; ++j) {
            if (j < nr) {
                const bool has_down = j < down;
                const bool has_up = j > 0 || !top;
                uint32_t cur[K], nxt[K];
                constexpr uint32_t SC = Acc::kScale;
                slot_pixels<Pix, K, FULL, PACKED, SC>(ring[j], c, W, cur);
                slot_pixels<Pix, K, FULL, PACKED, SC>(ring[j + 1], c, W, nxt);
                const uint32_t er0 = (uint32_t)__builtin_amdgcn_readlane((int)erv, j);
                const uint32_t er1 = (uint32_t)__builtin_amdgcn_readlane((int)erv, j + 1);
                uint32_t e0 = ((FULL || c + K < W) ? er0 : 0u) * SC;
                uint32_t e1 = ((FULL || c + K < W) ? er1 : 0u) * SC;
                uint32_t l1 = (NB == 8 ? (uint32_t)__builtin_amdgcn_readlane((int)elv, j + 1) : 0u) * SC;
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
                if constexpr (std::is_same<typename Acc::P, uint32_t>::value) {
                    row_pairs<NB, K, FULL>(cur, nxt, e0, e1, l1, has_up, has_down, c, W, acc);
                } else {
                    typename Acc::P pc[K], pn[K];
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        pc[k] = Acc::prep(cur[k]);
                        pn[k] = Acc::prep(nxt[k]);
                    }
                    row_pairs<NB, K, FULL>(pc, pn, Acc::prep(e0), Acc::prep(e1), Acc::prep(l1), has_up, has_down,
                                           c, W, acc);
                }
                if constexpr (Acc::kSpill) {
                    if (__any(acc.needs_spill())) row_pairs<NB, K, FULL>(cur, nxt, e0, e1, l1, has_up, has_down, c, W, spill);
                    acc.dmax = 0;
                }
            }
        }
    }
}

// Rows [r0, r1) of strip s of one image, by one wave.
template <typename Pix, int NB, int K, bool CLAMP, class Acc, class Spill>
__device__ __forceinline__ void strip_range(const KImage &im, int s, int64_t r0, int64_t r1, uint32_t Mm1,
                                            Acc &acc, Spill &spill, uint32_t &vmax) {
    constexpr bool kPk = pk_form<Pix, NB, K, CLAMP, Acc>();
    switch (strip_path(s, K, im.W, im.vec_ok != 0, kPk)) {
        case PATH_PK:
            if constexpr (kPk) pk_rows(im, s, r0, r1, acc, spill);
            break;
        case PATH_FULL_PACKED: strip_rows<Pix, NB, K, CLAMP, true, true>(im, s, r0, r1, Mm1, acc, spill, vmax); break;
        case PATH_FULL_ELEM: strip_rows<Pix, NB, K, CLAMP, true, false>(im, s, r0, r1, Mm1, acc, spill, vmax); break;
        case PATH_LAST_PACKED: strip_rows<Pix, NB, K, CLAMP, false, true>(im, s, r0, r1, Mm1, acc, spill, vmax); break;
        default: strip_rows<Pix, NB, K, CLAMP, false, false>(im, s, r0, r1, Mm1, acc, spill, vmax); break;
    }
}

// Units [la, lb) of one image (image-local, strip-major), by one wave.
template <typename Pix, int NB, int K, bool CLAMP, class Acc, class Spill>
__device__ __forceinline__ void wave_units(const KImage &im, int64_t la, int64_t lb, uint32_t Mm1, Acc &acc,
                                           Spill &spill, uint32_t &vmax) {
    int64_t u = la;
    while (u < lb) {
        const int s = (int)(u / im.H);
        const int64_t r = u - (int64_t)s * im.H;
        const int64_t rend = min(im.H, r + (lb - u));
        strip_range<Pix, NB, K, CLAMP>(im, s, r, rend, Mm1, acc, spill, vmax);
        u += rend - r;
    }
}

// ------------------------------------------------------------------------------------------------
// histograms -> difference arrays -> global accumulators

// Adds (d1, e) of grey level v. Packed mode: one int64 word per level holds E * 2^32 + D1 (exact
// while |sum D1| and |sum E| stay below 2^31, which the host guarantees by image size); otherwise
// D1 and E have a word each. Returns the old value(s) so that the caller can wait for completion.
__device__ __forceinline__ uint64_t add_levels(int64_t *acc, int M, bool packed, int v, int64_t d1, int64_t e) {
    unsigned long long *a = reinterpret_cast<unsigned long long *>(acc);
    uint64_t r = 0;
    if (packed) {
        const uint64_t w = ((uint64_t)e << 32) + (uint64_t)d1;
        if (w != 0) r = add_shared(a + v, w);
    } else {
        if (d1 != 0) r = add_shared(a + v, (uint64_t)d1);
        if (e != 0) r ^= add_shared(a + M + v, (uint64_t)e);
    }
    return r;
}

// E[v] for v >= 1 from the marginals at v-1: hmin + hmax - hsum[2v-3] - 2 hsum[2v-2] - hsum[2v-1].
__device__ __forceinline__ int64_t second_diff(int64_t lohi, const lds_u32 *hsum, int v, int M, int st = 1) {
    const int s = 2 * v - 2;
    int64_t e = lohi - 2 * (int64_t)hsum[s * st];
    if (s >= 1) e -= hsum[(s - 1) * st];
    if (s + 1 <= 2 * M - 2) e -= hsum[(s + 1) * st];
    return e;
}

// Sums of LDS words whose addresses follow from an index i in [i0, i1] (inclusive): `addr(i)` gives
// the word. Loads are issued 16 at a time before any is added (the index is clamped to the range,
// so every address is valid, and the surplus is dropped), so a sum of n words costs about n / 16 LDS
// round trips instead of n / 4.
constexpr int kLdsBatch = 16;
template <class Addr>
__device__ __forceinline__ uint32_t lds_sum(const lds_u32 *tab, int i0, int i1, Addr addr) {
    uint32_t acc = 0;
    for (int i = i0; i <= i1; i += kLdsBatch) {
        uint32_t t[kLdsBatch];
#pragma unroll
        for (int j = 0; j < kLdsBatch; ++j) t[j] = tab[addr(min(i + j, i1))];
#pragma unroll
        for (int j = 0; j < kLdsBatch; ++j) acc += (i + j <= i1) ? t[j] : 0u;
    }
    return acc;
}

// The C words of one cell of the banded table, loaded at once (16 bytes for four copies).
template <int C>
struct CellVec;
template <>
struct CellVec<1> {
    typedef uint32_t T;
    __device__ static __forceinline__ uint32_t sum(T v) { return v; }
};
template <>
struct CellVec<2> {
    typedef u32x2 T;
    __device__ static __forceinline__ uint32_t sum(T v) { return v.x + v.y; }
};
template <>
struct CellVec<4> {
    typedef u32x4 T;
    __device__ static __forceinline__ uint32_t sum(T v) { return (v.x + v.y) + (v.z + v.w); }
};

// Sum over all copies of n cells STEP cells apart, starting at cell `first` of the banded table (C
// copies interleaved). n must be the same for every lane of the wave (a per-lane trip count makes
// the compiler wait for each load before the next): eight loads are issued, then added, and each
// is one instruction with an immediate offset (STEP is a compile-time stride).
template <int STEP, int C>
__device__ __forceinline__ uint32_t lds_cells(const lds_u32 *tab, int first, int n) {
    typedef typename CellVec<C>::T V;
    const KOHLER_LDS V *q = reinterpret_cast<const KOHLER_LDS V *>(tab) + first;
    uint32_t acc = 0;
    int k = 0;
    for (; k + 8 <= n; k += 8, q += 8 * STEP) {
        V t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = q[j * STEP];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += CellVec<C>::sum(t[j]);
    }
    for (; k < n; ++k, q += STEP) acc += CellVec<C>::sum(q[0]);
    return acc;
}

// Projects the banded tables (all copies) on the three marginals and adds the workgroup's D1 and E
// to the image's accumulators. With S = kRowStride, cell (d, lo) is cell index d S + lo (its C copies
// are the words C (d S + lo) .. C (d S + lo) + C - 1):
//   hmin[v] = sum over d = 1..nb+1 of cell (d, v)   (row nb+1: the low values of the large gaps)
//   hmax[v] = sum over d = 1..nb of cell (d, v - d), plus the large gaps' own hmax
//   hsum[s] = sum over d = 1..nb with d = s (mod 2) of cell (d, (s - d) / 2), plus theirs
// Column v of hmin and the diagonals of hmax and hsum step by S, S - 1 and 2S - 1 cells, with the same
// number of terms for every level: a cell (d, lo) with lo + d > 255 is never written (no pair has
// it), and neither is a row's cell 256 .. S - 1, so the terms with d > v (hmax) or d > s (hsum), which
// land there ((d, v - d) is cell (d - 1) S + (S + v - d) of the row above), add zeros. hmin is written
// over the first word of its large-gap cell, hmax and hsum over the large-gap tables: each of those
// words is read only by the task that writes it.
template <int C>
__device__ __forceinline__ uint64_t merge_band_c(const KParams &p, lds_u32 *lds, int64_t *acc) {
    const int M = p.M, nb = p.band;
    constexpr int S = kRowStride;
    lds_u32 *tab = lds, *smax = lds + C * (nb + 2) * S, *ssum = smax + 256;
    const int gap_row = (nb + 1) * S;  // first cell of the large-gap row
    for (int x = threadIdx.x; x < 4 * M - 1; x += blockDim.x) {
        if (x < M) {
            const int v = x;
            const uint32_t h = lds_cells<S, C>(tab, S + v, nb + 1);
            tab[(gap_row + v) * C] = h;
        } else if (x < 2 * M) {
            const int v = x - M;
            smax[v] += lds_cells<S - 1, C>(tab, S + v - 1, nb);
        } else {
            const int sv = x - 2 * M;
            const int d0 = 2 - (sv & 1);  // the smallest gap with the parity of sv
            // nb / 2 terms for either parity, and for an odd band one more (d = nb) for odd s
            uint32_t h = lds_cells<2 * S - 1, C>(tab, d0 * S + (sv - d0) / 2, nb / 2);
            if ((nb & 1) && (sv & 1)) h += lds_cells<1, C>(tab, nb * S + (sv - nb) / 2, 1);
            ssum[sv] += h;
        }
    }
    __syncthreads();
    phase_stamp(3);
    uint64_t sink = 0;
    for (int v = threadIdx.x; v < M; v += blockDim.x) {
        const int64_t hmin = tab[(gap_row + v) * C], hmin1 = v >= 1 ? (int64_t)tab[(gap_row + v - 1) * C] : 0;
        const int64_t d1 = hmin - (int64_t)smax[v];
        const int64_t e = v >= 1 ? second_diff(hmin1 + smax[v - 1], ssum, v, M) : 0;
        sink ^= add_levels(acc, M, p.packed_acc != 0, v, d1, e);
    }
    return sink;
}

__device__ __forceinline__ uint64_t merge_band(const KParams &p, lds_u32 *lds, int64_t *acc) {
    if (p.copies == 4) return merge_band_c<4>(p, lds, acc);
    if (p.copies == 2) return merge_band_c<2>(p, lds, acc);
    return merge_band_c<1>(p, lds, acc);
}

// Project the triangular table onto hmax (row sums without the diagonal), hmin (column sums below
// the diagonal) and hsum (anti-diagonal sums without the diagonal). Thread task v < M: row v and
// column v (M - 1 reads); thread task M + s: anti-diagonals s and 2M - 2 - s (about s reads).
__device__ __forceinline__ uint64_t merge_tri(const KParams &p, lds_u32 *lds, int64_t *acc) {
    const int M = p.M;
    const lds_u32 *tab = lds;
    lds_u32 *hmin = lds + tri_words((uint32_t)M) + 64, *hmax = hmin + M, *hsum = hmax + M;
    // anti-diagonal s: (hi, lo) = (s - lo, lo) for lo from max(0, s - M + 1) to (s - 1) / 2
    auto anti = [&](int s) -> uint32_t {
        if (s < 1) return 0u;
        const int lo0 = max(0, s - M + 1), lo1 = (s - 1) / 2;
        return lds_sum(tab, lo0, lo1, [&](int lo) { return (int)tri_words((uint32_t)(s - lo)) + lo; });
    };
    for (int x = threadIdx.x; x < 2 * M; x += blockDim.x) {
        if (x < M) {
            const int v = x;
            const int rb = (int)tri_words((uint32_t)v);  // row v: lo = 0 .. v - 1
            hmax[v] = lds_sum(tab, 0, v - 1, [&](int lo) { return rb + lo; });
            // column v: rows h = v + 1 .. M - 1
            hmin[v] = lds_sum(tab, v + 1, M - 1, [&](int h) { return (int)tri_words((uint32_t)h) + v; });
        } else {
            const int s = x - M, s2 = 2 * M - 2 - s;
            hsum[s] = anti(s);
            if (s2 != s) hsum[s2] = anti(s2);
        }
    }
    __syncthreads();
    phase_stamp(3);
    uint64_t sink = 0;
    for (int v = threadIdx.x; v < M; v += blockDim.x) {
        const int64_t d1 = (int64_t)hmin[v] - (int64_t)hmax[v];
        const int64_t e = v >= 1 ? second_diff((int64_t)hmin[v - 1] + hmax[v - 1], hsum, v, M) : 0;
        sink ^= add_levels(acc, M, p.packed_acc != 0, v, d1, e);
    }
    return sink;
}

__device__ __forceinline__ uint64_t merge_marg(const KParams &p, lds_u32 *lds, int64_t *acc) {
    const int M = p.M, C = p.copies;
    if (C > 1) {
        // the copies of each entry summed into its first word (every entry by one thread)
        for (int j = threadIdx.x; j < 4 * M; j += blockDim.x) {
            uint32_t sum = 0;
            for (int c = 0; c < C; ++c) sum += lds[j * C + c];
            lds[j * C] = sum;
        }
        __syncthreads();
    }
    const lds_u32 *hmin = lds, *hdeg = lds + M * C, *hsum = lds + 2 * M * C;
    phase_stamp(3);
    uint64_t sink = 0;
    for (int v = threadIdx.x; v < M; v += blockDim.x) {
        const int64_t d1 = 2 * (int64_t)hmin[v * C] - (int64_t)hdeg[v * C];
        const int64_t e = v >= 1 ? second_diff((int64_t)hdeg[(v - 1) * C], hsum, v, M, C) : 0;
        sink ^= add_levels(acc, M, p.packed_acc != 0, v, d1, e);
    }
    return sink;
}

// ------------------------------------------------------------------------------------------------
// Wave-wide primitives for the one-wave finalize (all 64 lanes active)

// The int64 value of the lane selected by DPP control CTRL (rows outside ROW_MASK, and lanes whose
// source is outside their row, read 0).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the wave: shifts by 1, 2, 4 and 8 inside each row of 16 lanes, then row
// 0's total into row 1 and row 2's into row 3, then the first 32 lanes' total into rows 2 and 3.
__device__ __forceinline__ int64_t wave_iscan(int64_t v) {
    uint64_t x = (uint64_t)v;
    x += dpp64<0x111, 0xF>(x);  // row_shr:1
    x += dpp64<0x112, 0xF>(x);  // row_shr:2
    x += dpp64<0x114, 0xF>(x);  // row_shr:4
    x += dpp64<0x118, 0xF>(x);  // row_shr:8
    x += dpp64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return (int64_t)x;
}

// Running maximum over the wave (same pattern; 0 is the identity for the unsigned values used).
__device__ __forceinline__ uint64_t wave_imax(uint64_t x) {
    x = max(x, dpp64<0x111, 0xF>(x));
    x = max(x, dpp64<0x112, 0xF>(x));
    x = max(x, dpp64<0x114, 0xF>(x));
    x = max(x, dpp64<0x118, 0xF>(x));
    x = max(x, dpp64<0x142, 0xA>(x));
    x = max(x, dpp64<0x143, 0xC>(x));
    return x;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Lane l receives lane l-1's value; lane 0 receives 0.
__device__ __forceinline__ int64_t prev_lane64(int64_t x) {
    const uint32_t lo = from_prev_lane((uint32_t)(uint64_t)x, 0u);
    const uint32_t hi = from_prev_lane((uint32_t)((uint64_t)x >> 32), 0u);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Set lanes of `mask` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ------------------------------------------------------------------------------------------------
// Finalize for M <= 256: prefix sums, C, local maxima and t0 for the image with output index i, by
// the workgroup's first four waves (wave w, lane l owns threshold t = 64 w + l); the other waves only
// take part in the barriers.
//
// Local maxima: a run of equal C values starting at t (t = 0, or C(t) > C(t-1)) with C(t) > 0 is a
// local maximum when the first change of C after t is a fall, or there is none before M.
// Comparisons of neighbouring C values use the doubles: the division rounds correctly, so it is
// monotone, and two different doubles order their exact values the same way; equal doubles of a
// positive C are settled exactly (128-bit cross products). t0: the largest double marks every t
// with the exact largest C (and maybe others that round to it); a tie between several t is settled
// exactly, keeping the smallest t.

constexpr int kFinWaves = 4;
constexpr int kFinMaxM = 64 * kFinWaves;

struct FinScratch {
    int64_t tot[kFinWaves][3];  // per wave: sums of D1, E and v * E over its levels
    uint64_t ne[kFinWaves];     // per wave: levels where C changes (C(t) != C(t-1))
    uint64_t fa[kFinWaves];     // per wave: levels where C falls
    uint64_t cmax[kFinWaves];   // per wave: largest C as bits (C >= 0, so bits order as values)
    uint64_t mx[kFinWaves];     // per wave: local maxima
    uint64_t cand[kFinWaves];   // per wave: levels whose C equals the largest double
    int64_t sm[kFinMaxM], cnt[kFinMaxM];  // the curve, for the rare exact tie-break of t0
};

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }

// Lane l receives lane l-1's double; lane 0 receives 0.
__device__ __forceinline__ double prev_lane_f64(double x) {
    return __longlong_as_double(prev_lane64((int64_t)dbits(x)));
}

__device__ __forceinline__ void finalize_small(const KParams &p, int i, lds_u32 *lds) {
    const int M = p.M, R = p.nrep;
    const int lane = threadIdx.x & 63;
    const int w = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool active = w < kFinWaves;  // wave-uniform
    const int t = 64 * w + lane;
    const bool in = active && t < M;
    const int64_t RS = p.rep_stride;
    const bool packed = p.packed_acc != 0;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(p.acc + (int64_t)i * p.acc_stride);
    KOHLER_LDS FinScratch &fs = *reinterpret_cast<KOHLER_LDS FinScratch *>(lds);

    // 1. D1 and E of level t: the sum of the replicas (all loads issued before any is used), then
    //    the words are cleared for the next launch
    int64_t d1 = 0, e = 0;
    uint32_t rf = 0;
    if (active) {
        const int tt = in ? t : 0;
        // rounds of kGather loads, issued together (replica indices past R re-read the last one and
        // are dropped): one memory latency per round, and a single round for R <= kGather
        constexpr int kGather = 8;
        uint64_t s0 = 0, s1 = 0;
        // the range flag is read by every lane of the wave with the replicas (a single-lane load
        // would be waited for inside its branch) and used only at the end
        rf = __hip_atomic_load(gptr(p.rflag + i), __ATOMIC_RELAXED, KOHLER_XSCOPE);
        for (int rb = 0; rb < R; rb += kGather) {
            uint64_t v[kGather];
#pragma unroll
            for (int j = 0; j < kGather; ++j) v[j] = load_shared(acc + min(rb + j, R - 1) * RS + tt);
#pragma unroll
            for (int j = 0; j < kGather; ++j) s0 += rb + j < R ? v[j] : 0ull;
        }
        if (!packed) {  // images with 2^30 or more pairs: E has words of its own
            for (int rb = 0; rb < R; rb += kGather) {
                uint64_t v[kGather];
#pragma unroll
                for (int j = 0; j < kGather; ++j) v[j] = load_shared(acc + min(rb + j, R - 1) * RS + M + tt);
#pragma unroll
                for (int j = 0; j < kGather; ++j) s1 += rb + j < R ? v[j] : 0ull;
            }
        }
        if (in) {
            for (int r = 0; r < R; ++r) {
                store_shared(acc + r * RS + t, 0);
                if (!packed) store_shared(acc + r * RS + M + t, 0);
            }
        }
        if (packed) {
            // E * 2^32 + D1 summed as one word: |D1| < 2^31 because the image has < 2^30 pairs
            d1 = (int64_t)(int32_t)(uint32_t)s0;
            e = (int64_t)(s0 - (uint64_t)d1) >> 32;
        } else {
            d1 = (int64_t)s0;
            e = (int64_t)s1;
        }
        if (!in) d1 = e = 0;
    }
    phase_stamp(6);

    // 2. count = prefix of D1; with P0 = prefix of E and P1 = prefix of v E, sum(t) = (t+1) P0 - P1
    const int64_t x0 = wave_iscan(d1), x1 = wave_iscan(e), x2 = wave_iscan((int64_t)t * e);
    if (active && lane == 63) {
        fs.tot[w][0] = x0;
        fs.tot[w][1] = x1;
        fs.tot[w][2] = x2;
    }
    __syncthreads();
    clock_stamp(12);
    int64_t c0 = 0, c1 = 0, c2 = 0;  // totals of the waves before this one
    for (int v = 0; v < w && v < kFinWaves; ++v) {
        c0 += fs.tot[v][0];
        c1 += fs.tot[v][1];
        c2 += fs.tot[v][2];
    }
    const int64_t cnt = c0 + x0;
    const int64_t sm = (int64_t)(t + 1) * (c1 + x1) - (c2 + x2);
    const double C = cnt ? (double)sm / (double)cnt : 0.0;

    // 3. sign of C(t) - C(t-1): the previous level from the previous lane, or for lane 0 from the
    //    totals of the earlier waves (level 64 w - 1)
    int64_t ps = prev_lane64(sm), pk = prev_lane64(cnt);
    double pC = prev_lane_f64(C);
    if (lane == 0) {
        ps = (int64_t)(64 * w) * c1 - c2;
        pk = c0;
        pC = pk ? (double)ps / (double)pk : 0.0;
    }
    int rel = 0;
    if (in && t > 0) {
        rel = C > pC ? 1 : (C < pC ? -1 : 0);
        if (rel == 0 && sm != 0) rel = cmp_curve(sm, cnt, ps, pk);  // equal doubles: exact order
    }
    const uint64_t NE = __ballot(rel != 0), FA = __ballot(rel < 0);
    const bool start = in && sm > 0 && (t == 0 || rel > 0);
    const uint64_t cmax_w = readlane64(wave_imax(in ? dbits(C) : 0ull), 63);
    if (active && lane == 0) {
        fs.ne[w] = NE;
        fs.fa[w] = FA;
        fs.cmax[w] = cmax_w;
    }
    if (in) {
        fs.sm[t] = sm;
        fs.cnt[t] = cnt;
    }
    __syncthreads();
    clock_stamp(13);

    // 4. local maxima: the first change after t, in this wave or in a later one
    int next = -1;  // 1: fall, 0: rise, -1: no change before M
    const uint64_t later = lane == 63 ? 0ull : NE & (~0ull << (lane + 1));
    if (later) {
        next = (int)((FA >> __builtin_ctzll(later)) & 1ull);
    } else {
        for (int v = w + 1; v < kFinWaves; ++v) {
            const uint64_t nv = fs.ne[v];
            if (nv) {
                next = (int)((fs.fa[v] >> __builtin_ctzll(nv)) & 1ull);
                break;
            }
        }
    }
    const bool is_max = start && next != 0;
    const uint64_t MX = __ballot(is_max);
    uint64_t cmax = 0;
#pragma unroll
    for (int v = 0; v < kFinWaves; ++v) cmax = max(cmax, fs.cmax[v]);
    const uint64_t CA = __ballot(in && cmax != 0 && dbits(C) == cmax);
    if (active && lane == 0) {
        fs.mx[w] = MX;
        fs.cand[w] = CA;
    }
    __syncthreads();
    clock_stamp(14);

    // 5. compaction of the maxima in ascending order, and t0
    uint32_t below = 0, found = 0, ncand = 0;
#pragma unroll
    for (int v = 0; v < kFinWaves; ++v) {
        const uint32_t nv = (uint32_t)__builtin_popcountll(fs.mx[v]);
        below += v < w ? nv : 0u;
        found += nv;
        ncand += (uint32_t)__builtin_popcountll(fs.cand[v]);
    }
    int32_t *othr = p.thr + (int64_t)i * p.thr_stride;
    if (is_max) {
        const uint32_t pos = below + lanes_below(MX);
        if ((int64_t)pos < (int64_t)p.cap) othr[pos] = t;
    }
    if (in) {
        p.sum[(int64_t)i * p.ostride + t] = sm;
        p.count[(int64_t)i * p.ostride + t] = cnt;
        p.C[(int64_t)i * p.ostride + t] = C;
    }
    if (w == 0 && lane == 0) {
        int32_t t0 = -1;
        int64_t bs_ = 0, bk_ = 0;
        for (int v = 0; v < kFinWaves; ++v) {
            for (uint64_t m = fs.cand[v]; m; m &= m - 1) {
                const int tc = 64 * v + __builtin_ctzll(m);
                if (t0 < 0) {
                    t0 = tc;
                    bs_ = fs.sm[tc];
                    bk_ = fs.cnt[tc];
                    if (ncand == 1) break;
                } else if (cmp_curve(fs.sm[tc], fs.cnt[tc], bs_, bk_) > 0) {
                    t0 = tc;
                    bs_ = fs.sm[tc];
                    bk_ = fs.cnt[tc];
                }
            }
        }
        __hip_atomic_store(gptr(p.rflag + i), 0u, __ATOMIC_RELAXED, KOHLER_XSCOPE);
        store_shared(p.done + i, 0);
        p.n_thr[(int64_t)i * p.istride] = (int32_t)found;
        p.t0[(int64_t)i * p.istride] = t0;
        p.status[(int64_t)i * p.istride] = rf ? ST_RANGE : ((int64_t)found > (int64_t)p.cap ? ST_CAPACITY : ST_OK);
    }
    phase_stamp(7);
}

// ------------------------------------------------------------------------------------------------
// finalize: prefix sums, C, local maxima and t0 for the image with output index i (run by one
// workgroup)
//
// LDS use (the histogram tables are dead by now): one byte per threshold from address 0: bits 0-1 =
// sign of C(t) - C(t-1) (0 equal, 1 rise, 2 fall), bit 2 = C(t) > 0; from fin_gather_offset the
// replica sums of the levels (packed accumulators).

// Exclusive prefix sums of three values over the workgroup (all threads, blockDim.x a multiple of 64,
// at most 1024), and their totals; the barriers order LDS only, so global stores issued before stay
// in flight.
__device__ __forceinline__ void block_exscan3(int64_t (&x)[3], LdsScratch &bs, int64_t (&total)[3]) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t inc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) inc[q] = wave_iscan(x[q]);
    if (lane == 63) {
        bs.scan[wid] = inc[0];
        bs.red_s[wid] = inc[1];
        bs.red_k[wid] = inc[2];
    }
    lds_barrier();
    int64_t before[3] = {0, 0, 0}, all[3] = {0, 0, 0};
    for (int w = 0; w < nw; ++w) {
        const int64_t a = bs.scan[w], b = bs.red_s[w], c = bs.red_k[w];
        if (w < wid) {
            before[0] += a;
            before[1] += b;
            before[2] += c;
        }
        all[0] += a;
        all[1] += b;
        all[2] += c;
    }
    lds_barrier();  // every wave has read the totals before the scratch is written again
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        x[q] = before[q] + inc[q] - x[q];
        total[q] = all[q];
    }
}

// The finishing step for M > 256 (the whole workgroup): thread j takes the L = ceil(M / blockDim)
// consecutive levels [j L, j L + L). One pass forms its totals of D1, E and v E, one workgroup scan
// gives the prefixes before its levels, a second pass gives count, sum and C of each level and the
// sign of C(t) - C(t - 1) (the level before its first comes from the prefix itself); the local
// maxima are counted per thread and placed in ascending order by a second scan.
__device__ __forceinline__ void finalize(const KParams &p, int i, lds_u32 *lds, LdsScratch &bs) {
    const int M = p.M, tid = threadIdx.x, nt = blockDim.x;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(p.acc + (int64_t)i * p.acc_stride);
    const int R = p.nrep;
    const int64_t RS = p.rep_stride;
    int64_t *osum = p.sum + (int64_t)i * p.ostride;
    int64_t *ocnt = p.count + (int64_t)i * p.ostride;
    double *oC = p.C + (int64_t)i * p.ostride;
    KOHLER_LDS uint8_t *flags = reinterpret_cast<KOHLER_LDS uint8_t *>(lds);  // M bytes
    // the replica sums of every level (packed accumulators), gathered before the scans
    KOHLER_LDS uint64_t *gsum = reinterpret_cast<KOHLER_LDS uint64_t *>(
        reinterpret_cast<KOHLER_LDS uint8_t *>(lds) + fin_gather_offset(M, nt));
    const bool packed = p.packed_acc != 0;

    // the range flag is fetched now, with the accumulators, and used at the very end
    uint32_t rf = 0;
    if (tid == 0) rf = __hip_atomic_load(gptr(p.rflag + i), __ATOMIC_RELAXED, KOHLER_XSCOPE);
    phase_stamp(6);
    // this thread's levels [lo, hi)
    const int L = (M + nt - 1) / nt;
    const int lo = min(M, tid * L), hi = min(M, lo + L);

    // Packed accumulators: every level's replica sum into LDS first, kFinGather levels per thread
    // with all their loads in flight (indices clamped, the surplus dropped): about R / 2 memory
    // latencies in all.
    if (packed) {
        constexpr int kFinGather = 8;
        for (int b = 0; b < M; b += kFinGather * nt) {
            uint64_t sum[kFinGather];
#pragma unroll
            for (int k = 0; k < kFinGather; ++k) sum[k] = 0;
            for (int r = 0; r < R; r += 2) {  // two replicas per round (the second clamped, dropped past R)
                const int r2 = min(r + 1, R - 1);
                uint64_t v[kFinGather], w[kFinGather];
#pragma unroll
                for (int k = 0; k < kFinGather; ++k) {
                    v[k] = load_shared(acc + r * RS + min(b + k * nt + tid, M - 1));
                    w[k] = load_shared(acc + r2 * RS + min(b + k * nt + tid, M - 1));
                }
#pragma unroll
                for (int k = 0; k < kFinGather; ++k) sum[k] += v[k] + (r + 1 < R ? w[k] : 0ull);
            }
#pragma unroll
            for (int k = 0; k < kFinGather; ++k) {
                const int t = b + k * nt + tid;
                if (t < M) gsum[(t % L) * nt + t / L] = sum[k];  // level j L + q of thread j at q nt + j
            }
        }
        lds_barrier();
    }
    // D1 and E of level t: from the gathered sums (E * 2^32 + D1 in one word, |D1| < 2^31 because
    // the image has < 2^30 pairs), else summed from the replicas' two words (images with 2^30 or
    // more pairs)
    auto level = [&](int t, int64_t &d1, int64_t &e) {
        if (packed) {
            const uint64_t w = gsum[(t - lo) * nt + tid];  // consecutive threads, consecutive words
            d1 = (int64_t)(int32_t)(uint32_t)w;
            e = (int64_t)(w - (uint64_t)d1) >> 32;
        } else {
            uint64_t w0 = 0, w1 = 0;
            for (int r = 0; r < R; ++r) {
                w0 += load_shared(acc + r * RS + t);
                w1 += load_shared(acc + r * RS + M + t);
            }
            d1 = (int64_t)w0;
            e = (int64_t)w1;
        }
    };

    // 1. this thread's totals, then the prefixes before its levels. With P0(t) = sum_{v<=t} E[v]
    //    and P1(t) = sum_{v<=t} v E[v], the double prefix sum of E is sum(t) = (t + 1) P0(t) - P1(t)
    //    (int64 arithmetic wraps, but the result is exact because sum(t) itself fits).
    int64_t x[3] = {0, 0, 0}, tot[3];
    for (int t = lo; t < hi; ++t) {
        int64_t d1, e;
        level(t, d1, e);
        x[0] += d1;
        x[1] += e;
        x[2] += (int64_t)t * e;
    }
    block_exscan3(x, bs, tot);

    // 2. count, sum and C per level; flags: bit 0 rise, bit 1 fall (against level t - 1), bit 2 C > 0
    //    Orders are taken on the rounded C first: rounding is monotonic, so different doubles
    //    order the exact quotients the same way; equal doubles are settled by the exact compare.
    int64_t cnt = x[0], P0 = x[1], P1 = x[2];
    int64_t ps = (int64_t)lo * P0 - P1, pk = cnt;  // level lo - 1
    double pC = pk ? (double)ps / (double)pk : 0.0;
    int32_t bt = -1;
    int64_t bsum = 0, bcnt = 0;
    double bC = 0.0;
    for (int t = lo; t < hi; ++t) {
        int64_t d1, e;
        level(t, d1, e);
        cnt += d1;
        P0 += e;
        P1 += (int64_t)t * e;
        const int64_t sm = (int64_t)(t + 1) * P0 - P1;
        const double C = cnt ? (double)sm / (double)cnt : 0.0;
        osum[t] = sm;
        ocnt[t] = cnt;
        oC[t] = C;
        int r = 0;
        if (t > 0) {
            r = C > pC ? 1 : (C < pC ? -1 : 0);
            if (r == 0) r = cmp_curve(sm, cnt, ps, pk);
        }
        const bool pos = cnt > 0 && sm > 0;  // C(t) > 0
        flags[t] = (uint8_t)((r > 0 ? 1 : (r < 0 ? 2 : 0)) | (pos ? 4 : 0));
        if (bt < 0 || C > bC || (C == bC && cmp_curve(sm, cnt, bsum, bcnt) > 0)) {
            bt = t;
            bsum = sm;
            bcnt = cnt;
            bC = C;
        }
        ps = sm;
        pk = cnt;
        pC = C;
    }
    lds_barrier();
    clock_stamp(12);

    // 3. local maxima: a run start (t == 0 or a rise) with positive C whose run ends in a fall or
    //    at M; this thread's are written after those of the threads before it
    auto is_max = [&](int t) -> bool {
        const uint32_t f = flags[t];
        if (!((f & 4u) && (t == 0 || (f & 3u) == 1u))) return false;
        int u = t + 1;
        while (u < M && (flags[u] & 3u) == 0u) ++u;
        return u == M || (flags[u] & 3u) == 2u;
    };
    int64_t y[3] = {0, 0, 0}, ytot[3];
    for (int t = lo; t < hi; ++t) y[0] += is_max(t) ? 1 : 0;
    block_exscan3(y, bs, ytot);
    int32_t *othr = p.thr + (int64_t)i * p.thr_stride;
    int64_t posn = y[0];
    for (int t = lo; t < hi; ++t)
        if (is_max(t)) {
            if (posn < p.cap) othr[posn] = t;
            ++posn;
        }
    const int64_t found = ytot[0];
    clock_stamp(13);

    // 4. t0: smallest t attaining max C (each thread's candidate is the first maximum of its levels)
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
    lds_barrier();
    clock_stamp(14);
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
        __hip_atomic_store(gptr(p.rflag + i), 0u, __ATOMIC_RELAXED, KOHLER_XSCOPE);
        store_shared(p.done + i, 0);
        p.n_thr[(int64_t)i * p.istride] = (int32_t)found;
        p.t0[(int64_t)i * p.istride] = t0;
        p.status[(int64_t)i * p.istride] = rf ? ST_RANGE : (found > p.cap ? ST_CAPACITY : ST_OK);
    }
    // the replicas cleared for the next launch
    for (int t = tid; t < M; t += nt) {
        for (int r = 0; r < R; ++r) {
            store_shared(acc + r * RS + t, 0);
            if (!packed) store_shared(acc + r * RS + M + t, 0);
        }
    }
    phase_stamp(7);
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

// Output index of image i (used only on the error path, from one thread).
__device__ __forceinline__ int image_desc_out(const KParams &p, int i) {
    return p.n == 1 ? p.img0.out : gptr(p.imgs)[i].out;
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
        im.out = q->out;
    }
    im.ptr = (const void *)uniform64((int64_t)im.ptr);
    im.H = uniform64(im.H);
    im.W = uniform64(im.W);
    im.pitch = uniform64(im.pitch);
    im.ustart = uniform64(im.ustart);
    im.nunits = uniform64(im.nunits);
    im.nstrips = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)im.nstrips);
    im.vec_ok = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)im.vec_ok);
    im.out = (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)im.out);
    return im;
}

// Zeroes the first `words` (a multiple of 4) words of the workgroup's LDS and the chunk counter.
__device__ __forceinline__ void clear_lds(lds_u32 *lds, LdsScratch &bs, uint32_t words) {
    for (uint32_t x = threadIdx.x; x < words / 4; x += blockDim.x)
        reinterpret_cast<KOHLER_LDS u32x4 *>(lds)[x] = u32x4{0u, 0u, 0u, 0u};
    if (threadIdx.x == 0) bs.next = 0;
    lds_barrier();
    phase_stamp(1);
}

// After the pair work of `units` units of image im (of `expected` in the whole launch, counted in
// the ticket): range flag, merge into the image's accumulators, ticket, and the finalize step when
// this workgroup completed the image. Called by every thread of the workgroup.
template <int FORM, bool CLAMP>
__device__ __forceinline__ void flush_image(const KParams &p, lds_u32 *lds, LdsScratch &bs, const KImage &im,
                                            uint32_t vmax, int64_t units, int64_t expected) {
    const uint32_t Mm1 = (uint32_t)p.M - 1u;
    const int i = im.out;
    uint64_t sink = 0;
    if constexpr (CLAMP) {
        vmax = wave_max(vmax);
        if ((threadIdx.x & 63) == 0 && vmax > Mm1)
            sink = __hip_atomic_fetch_or(gptr(p.rflag + i), 1u, __ATOMIC_RELAXED, KOHLER_XSCOPE);
    }
    __syncthreads();
    phase_stamp(2);
    if (units == 0) return;  // uniform: nothing to add, and no ticket to take
    int64_t *acc_g = p.acc + (int64_t)i * p.acc_stride + (int64_t)(blockIdx.x % (uint32_t)p.nrep) * p.rep_stride;
    if constexpr (FORM == FORM_BAND) sink ^= merge_band(p, lds, acc_g);
    else if constexpr (FORM == FORM_TRI) sink ^= merge_tri(p, lds, acc_g);
    else sink ^= merge_marg(p, lds, acc_g);

    // every contribution of this workgroup has been performed once its returned value is here:
    // consuming the values makes the wave wait for all of them before the barrier
    asm volatile("" ::"v"((uint32_t)sink), "v"((uint32_t)(sink >> 32)));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    phase_stamp(4);
    if (threadIdx.x == 0) {
        const unsigned long long old = add_shared(p.done + i, (unsigned long long)units);
        bs.last = (old + (unsigned long long)units == (unsigned long long)expected) ? 1 : 0;
    }
    __syncthreads();
    phase_stamp(5);
    if (bs.last) {
        if constexpr (FORM == FORM_MARG) {
            if (p.M <= kFinMaxM) finalize_small(p, i, lds);
            else finalize(p, i, lds, bs);
        } else {
            finalize_small(p, i, lds);
        }
    }
    __syncthreads();
}

// Largest workgroup of an instance: 1024 threads where the registers fit four waves per SIMD without
// spilling, else 512 (the marginal form and the 8-neighbourhood with 8 pixels per lane).
template <int NB, int K, int FORM>
constexpr int max_block() { return (FORM == FORM_MARG || (NB == 8 && K == 8)) ? 512 : 1024; }

template <typename Pix, int NB, int K, int FORM, bool CLAMP>
__global__ void __launch_bounds__((max_block<NB, K, FORM>())) curve_kernel(KParams p) {
    extern __shared__ __align__(16) uint32_t lds_raw[];
    lds_u32 *lds = (lds_u32 *)lds_raw;
    LdsScratch &bs = *reinterpret_cast<LdsScratch *>(
        reinterpret_cast<KOHLER_LDS uint8_t *>(lds) + lds_main_bytes(FORM, p.M, p.band, (int)blockDim.x, p.copies));

    if ((uint32_t)(size_t)lds != 0u) {
        // the LDS layout assumption behind lds_at() does not hold: report, compute nothing
        if (blockIdx.x == 0 && threadIdx.x == 0)
            for (int i = 0; i < p.n; ++i) p.status[(int64_t)image_desc_out(p, i) * p.istride] = ST_LAYOUT;
        return;
    }
    phase_stamp(0);
    phase_place();
    const int G = gridDim.x;
    // consecutive logical workgroups land on the same XCD (the dispatcher deals blocks round-robin)
    const int g = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const uint32_t Mm1 = (uint32_t)p.M - 1u;

    uint32_t table_words;
    if constexpr (FORM == FORM_BAND)
        table_words = ((uint32_t)p.copies * ((uint32_t)p.band + 2u) * kRowStride + 768u + 3u) & ~3u;
    else if constexpr (FORM == FORM_TRI) table_words = (tri_words((uint32_t)p.M) + 64u + 3u) & ~3u;
    else table_words = 4u * (uint32_t)p.M * (uint32_t)p.copies;

    auto clear_tables = [&]() { clear_lds(lds, bs, table_words); };

    // Runs `chunks(acc, spill, vmax)` with the accumulators of this kernel's form; it must feed every
    // pair of the units the wave takes on.
    auto accumulate = [&](auto &&chunks) -> uint32_t {
        uint32_t vmax = 0;
        if constexpr (FORM == FORM_BAND) {
            const uint32_t nb = (uint32_t)p.band, rows = nb + 2u;
            const uint32_t lane = threadIdx.x & 63u, nc = (uint32_t)p.copies;
            const uint32_t cl = lane % nc, cn = ((lane + 1u) & 63u) % nc;  // copies of this lane and the next
            const uint16_t C16 = (uint16_t)nc, cap = (uint16_t)(nc * (nb + 1u));
            BandAcc acc{4u * (nb + 1u), nc, 4u * cl, 0u, u16x2{C16, C16}, u16x2{(uint16_t)cl, (uint16_t)cl},
                        u16x2{0, (uint16_t)(cl - cn)}, u16x2{cap, cap}, u16x2{0, 0}};
            const uint32_t spill0 = 4u * (uint32_t)p.copies * rows * kRowStride;
            SpillAcc spill{spill0, spill0 + 4u * 256u, nb};
            chunks(acc, spill, vmax, Mm1 * BandAcc::kScale);
            vmax /= BandAcc::kScale;
        } else if constexpr (FORM == FORM_TRI) {
            TriAcc acc{2u * tri_words((uint32_t)p.M), 0u, 0u};
            SpillAcc spill{0u, 0u, 0u};  // not used by the triangular form
            chunks(acc, spill, vmax, Mm1);
        } else {
            // lane l adds to copy l % copies (1 or 2) of each table
            const uint32_t nc = (uint32_t)p.copies, cl = (threadIdx.x & 63u) & (nc - 1u);
            const uint32_t Mc = (uint32_t)p.M * nc;
            MargAcc acc{lds + cl, lds + Mc + cl, lds + 2u * Mc + cl, 0u, 0u, nc == 2u ? 1u : 0u};
            SpillAcc spill{0u, 0u, 0u};  // not used by the marginal form
            chunks(acc, spill, vmax, Mm1);
        }
        phase_wave_stamp();
        return vmax;
    };

    auto flush = [&](const KImage &im, uint32_t vmax, int64_t units, int64_t expected) {
        flush_image<FORM, CLAMP>(p, lds, bs, im, vmax, units, expected);
    };

    // rows a wave processes at a time: a chunk of the single-image launch, a claim of the batched one
    constexpr int B = row_batch<Pix, NB, K, CLAMP>();
    // the single-image launch of the 8-bit packed instances deals chunks of one packed batch
    constexpr bool kPkKernel =
        FORM == FORM_BAND && std::is_same<Pix, uint8_t>::value && K == 8 && NB == 4 && !CLAMP;
    constexpr int BD = kPkKernel ? kPkRows : B;

    if (p.dyn) {
        // One image: a chunk is BD consecutive rows of one strip. Chunks are numbered row-block major
        // (chunk c covers strip c mod nstrips of row block c / nstrips), so neighbouring strips of
        // the same rows get consecutive numbers, and they are dealt round-robin to the workgroups
        // (chunk c to logical workgroup c mod G): every workgroup samples the whole image, costly
        // regions (many large-gap pairs) spread evenly, and the next strip's first column, which a
        // strip's rows also read, is fetched at about the same time by a workgroup on the same XCD
        // (shared L2). Waves claim their workgroup's chunks in turn, the last ones in half-chunk
        // pieces so that the waves finish closer together.
        const KImage im = image_desc(p, 0);
        const int64_t ns = im.nstrips;
        const int64_t nblocks = (im.H + BD - 1) / BD;
        const int64_t nchunks = nblocks * ns;
        // number of chunks c < n with c = g (mod G)
        auto upto = [&](int64_t n) -> int64_t { return n > g ? (n - g - 1) / G + 1 : 0; };
        const int64_t mine = upto(nchunks);  // chunks of this workgroup
        clear_tables();
        auto claim = [&]() -> uint32_t {
            uint32_t k = 0;
            if ((threadIdx.x & 63) == 0)
                k = __hip_atomic_fetch_add(&bs.next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return (uint32_t)__builtin_amdgcn_readfirstlane(k);
        };
        const uint32_t vmax = accumulate([&](auto &acc, auto &spill, uint32_t &vm, uint32_t mm1) {
            // chunk numbers stay below 2^32 (at most 2^40 pixels, chunks of at least 1024: B >= 4 rows
            // by 256 columns, or kPkRows >= 3 rows by 512), so the decode is a 32-bit division by a
            // wave-uniform value
            constexpr uint32_t kHalf = (uint32_t)BD / 2, kPieces = 2;
            const uint32_t ntail = (uint32_t)min<int64_t>(mine, (int64_t)(blockDim.x >> kTailShift));
            const uint32_t whole = (uint32_t)mine - ntail;
            const uint32_t nclaims = whole + ntail * kPieces;
            // strip and rows [r0, r1) of claim j (empty: a piece past the last row of a short final
            // row block)
            auto decode = [&](uint32_t j, int &strip, int64_t &r0, int64_t &r1) {
                uint32_t jc = j, off = 0, len = (uint32_t)BD;
                if (j >= whole) {
                    jc = whole + (j - whole) / kPieces;
                    off = ((j - whole) % kPieces) * kHalf;
                    len = off ? (uint32_t)BD - kHalf : kHalf;
                }
                const uint32_t c = (uint32_t)g + jc * (uint32_t)G;
                const uint32_t blk = c / (uint32_t)ns;
                strip = (int)(c - blk * (uint32_t)ns);
                r0 = (int64_t)blk * BD + off;
                r1 = min(im.H, r0 + (int64_t)len);
            };
            for (uint32_t j = claim(); j < nclaims; j = claim()) {
                int strip;
                int64_t r0, r1;
                decode(j, strip, r0, r1);
                if (r0 < r1) strip_range<Pix, NB, K, CLAMP>(im, strip, r0, r1, mm1, acc, spill, vm);
            }
        });
        // units of this workgroup: BD rows per chunk, less the short chunks of the last row block
        const int64_t last_rows = im.H - (nblocks - 1) * BD;
        const int64_t units = mine * BD - (upto(nchunks) - upto(nchunks - ns)) * (BD - last_rows);
        flush(im, vmax, units, im.nunits);
        return;
    }

    // Several images: each workgroup takes a contiguous range of the launch's unit space; inside an
    // image's part of it, waves claim chunks of B units from a workgroup counter.
    const int64_t U = p.total_units;
    int64_t u = (int64_t)g * U / G;
    const int64_t uend = (int64_t)(g + 1) * U / G;
    while (u < uend) {
        const int i = (p.n == 1) ? 0 : find_image(p, u);
        const KImage im = image_desc(p, i);
        const int64_t seg_end = min(uend, im.ustart + im.nunits);
        const int64_t nseg = seg_end - u;
        clear_tables();
        const int64_t lbase = u - im.ustart;
        const uint32_t nchunks = (uint32_t)((nseg + B - 1) / B);
        auto claim = [&]() -> uint32_t {
            uint32_t k = 0;
            if ((threadIdx.x & 63) == 0)
                k = __hip_atomic_fetch_add(&bs.next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            return (uint32_t)__builtin_amdgcn_readfirstlane(k);
        };
        const uint32_t vmax = accumulate([&](auto &acc, auto &spill, uint32_t &vm, uint32_t mm1) {
            for (uint32_t k = claim(); k < nchunks; k = claim()) {
                const int64_t ca = lbase + (int64_t)k * B, cb = min(lbase + nseg, ca + B);
                wave_units<Pix, NB, K, CLAMP>(im, ca, cb, mm1, acc, spill, vm);
            }
        });
        flush(im, vmax, nseg, im.nunits);
        u = seg_end;
    }
}

// ------------------------------------------------------------------------------------------------
// Other neighbourhoods and the pre-filtered image (NbParams): one image per launch. The image is cut
// into tiles of tile_rows x blockDim pixels, dealt round-robin to the workgroups. A tile's values
// (rows r0 .. r0 + tile_rows + radius - 1, columns c0 - radius .. c0 + blockDim + radius - 1, the
// ones a pair of its pixels can reach) are staged in LDS as 16-bit values, each read once from
// memory, or computed through the 3x3 binomial pre-filter; then every thread walks its column of
// the tile and adds, for each pixel, the pairs of its row's half offsets (Sec. 3.2 eqs (7)-(9):
// each unordered pair once) into the joint (triangular) or the marginal tables of the workgroup.

// One pixel of the image (element index y * pitch + x).
template <typename Pix>
__device__ __forceinline__ uint32_t image_px(const KImage &im, int64_t y, int64_t x) {
    return (uint32_t)gptr(static_cast<const Pix *>(im.ptr) + y * im.pitch)[(uint32_t)x];
}

// The 3x3 binomial low-pass at (y, x): weights 1 2 1 / 2 4 2 / 1 2 1, coordinates outside the image
// replaced by the nearest pixel of the image, (sum + 8) >> 4. `centre` receives f(y, x).
template <typename Pix>
__device__ __forceinline__ uint32_t binomial3_at(const KImage &im, int64_t y, int64_t x, uint32_t &centre) {
    const int64_t ys[3] = {y > 0 ? y - 1 : 0, y, y + 1 < im.H ? y + 1 : im.H - 1};
    const int64_t xs[3] = {x > 0 ? x - 1 : 0, x, x + 1 < im.W ? x + 1 : im.W - 1};
    uint32_t rows[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint32_t a = image_px<Pix>(im, ys[i], xs[0]), b = image_px<Pix>(im, ys[i], xs[1]),
                       c = image_px<Pix>(im, ys[i], xs[2]);
        if (i == 1) centre = b;
        rows[i] = a + 2u * b + c;
    }
    return (rows[0] + 2u * rows[1] + rows[2] + 8u) >> 4;
}

// Staging of a tile: rows y0 .. y0 + nrows - 1 and columns x0 .. x0 + ncols - 1 of the image (y0 >= -1,
// y0 < H, ncols at most twice the block) are loaded into registers, two column slots per thread and
// every row of a slot in flight together, while the previous tile's pairs are formed; then stored
// to LDS. Every address is clamped into the image. MODE: STAGE_MARK stores kNbOut for positions
// outside the image and clamps values to M - 1 (when CLAMP); STAGE_RAW stores the clamped position's
// pixel unchanged (the pre-filter's border). With CLAMP, vmax takes the tile's own pixels: rows
// own_r .. own_r + own_rows - 1 and columns own_c .. own_c + blockDim - 1, inside the image.
constexpr int kNbMaxStage = 16 + kNbMaxRadius + 2;  // rows of a staged region (tile rows <= 16)
enum StageMode { STAGE_MARK, STAGE_RAW };
// Tile value of a position outside the image (above any level: values are at most M - 1 <= 8191).
constexpr uint32_t kNbOut = 0xFFFFu;

struct StageRegs {
    uint32_t v[2][kNbMaxStage];
};

struct StageRegion {
    int64_t y0;
    int x0, nrows, ncols;
    int own_r, own_rows, own_c;
};

template <typename Pix>
__device__ __forceinline__ void load_region(const KImage &im, const StageRegion &g, StageRegs &sr) {
    const int64_t H = im.H;
    const int W = (int)im.W;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int rx = (int)threadIdx.x + j * (int)blockDim.x;
        if (rx < g.ncols) {
            const int x = g.x0 + rx;
            const int xc = x < 0 ? 0 : (x >= W ? W - 1 : x);
#pragma unroll
            for (int r = 0; r < kNbMaxStage; ++r) {
                if (r < g.nrows) {  // uniform; nothing but the load, so that no wait is needed here
                    const int64_t y = g.y0 + r;
                    sr.v[j][r] = image_px<Pix>(im, y < 0 ? 0 : (y >= H ? H - 1 : y), xc);
                }
            }
        }
    }
}

template <int MODE, bool CLAMP>
__device__ __forceinline__ void store_region(const KImage &im, const StageRegion &g, const StageRegs &sr,
                                             KOHLER_LDS uint16_t *dst, uint32_t mm1, uint32_t &vmax) {
    const int W = (int)im.W;
    const int TW = (int)blockDim.x;
    // rows of the region inside the image: [in0, in1)
    const int in0 = g.y0 < 0 ? 1 : 0;
    const int64_t hy = im.H - g.y0;
    const int in1 = hy < g.nrows ? (int)hy : g.nrows;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int rx = (int)threadIdx.x + j * TW;
        if (rx < g.ncols) {
            const int x = g.x0 + rx;
            const bool xin = x >= 0 && x < W;
            const bool own_x = xin && rx >= g.own_c && rx < g.own_c + TW;
#pragma unroll
            for (int r = 0; r < kNbMaxStage; ++r) {
                if (r < g.nrows) {
                    uint32_t v = sr.v[j][r];
                    if constexpr (CLAMP) {
                        if (own_x && r >= g.own_r && r < g.own_r + g.own_rows) vmax = max(vmax, v);
                    }
                    if constexpr (MODE == STAGE_MARK) {
                        if constexpr (CLAMP) v = min(v, mm1);
                        v = (xin && r >= in0 && r < in1) ? v : kNbOut;
                    }
                    dst[r * g.ncols + rx] = (uint16_t)v;
                }
            }
        }
    }
}

template <typename Pix, int FORM, bool CLAMP>
__global__ void __launch_bounds__(kNbBlock) nbhd_kernel(NbParams q) {
    extern __shared__ __align__(16) uint32_t lds_raw[];
    lds_u32 *lds = (lds_u32 *)lds_raw;
    const KParams &p = q.k;
    LdsScratch &bs = *reinterpret_cast<LdsScratch *>(reinterpret_cast<KOHLER_LDS uint8_t *>(lds) + q.bs_off);
    if ((uint32_t)(size_t)lds != 0u) {
        if (blockIdx.x == 0 && threadIdx.x == 0) p.status[(int64_t)p.img0.out * p.istride] = ST_LAYOUT;
        return;
    }
    phase_stamp(0);
    phase_place();
    const int G = gridDim.x;
    const int g = (G % 8 == 0) ? (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
    const uint32_t Mm1 = (uint32_t)p.M - 1u;
    const uint32_t table_words = FORM == FORM_TRI ? (tri_words((uint32_t)p.M) + 64u + 3u) & ~3u : 4u * (uint32_t)p.M;
    clear_lds(lds, bs, table_words);
    phase_stamp(1);

    const KImage im = image_desc(p, 0);
    const int64_t H = im.H, W = im.W;
    const int R = q.radius, TH = q.tile_rows, TW = (int)blockDim.x, TC = TW + 2 * R;
    KOHLER_LDS uint16_t *tile = reinterpret_cast<KOHLER_LDS uint16_t *>(reinterpret_cast<KOHLER_LDS uint8_t *>(lds) +
                                                                        q.tile_off);
    typedef typename std::conditional<FORM == FORM_TRI, TriAcc, MargAcc>::type Acc;
    Acc acc = [&]() {
        if constexpr (FORM == FORM_TRI) return TriAcc{2u * tri_words((uint32_t)p.M), 0u, 0u};
        else return MargAcc{lds, lds + p.M, lds + 2 * p.M, 0u, 0u};
    }();
    uint32_t vmax = 0;
    int64_t mine = 0;
    const int W32 = (int)W;  // W <= 2^30: columns are 32-bit; rows are counted from the tile's first
    KOHLER_LDS uint16_t *raw = reinterpret_cast<KOHLER_LDS uint16_t *>(reinterpret_cast<KOHLER_LDS uint8_t *>(lds) +
                                                                       q.raw_off);
    const int F = q.filter ? 1 : 0;
    // the half offsets as tile offsets dy TC + dx, one per lane (lane 16 par + a), read once and then
    // taken with a lane read by the wave-uniform index: indexing the argument with a loop variable
    // would read it from memory on every use
    const int lane = (int)(threadIdx.x & 63u);
    const int lpar = (lane >> 4) & 1, la = lane & 15;
    const int offv = (int)q.hdy[lpar][la] * TC + (int)q.hdx[lpar][la];
    const int na0 = q.nhalf[0], na1 = q.nhalf[1], na_max = max(na0, na1);
    [[maybe_unused]] const int nf0 = q.nfull[0], nf1 = q.nfull[1];
    // whole-neighbourhood offsets (degrees of the pixels near the border): a copy in LDS, per parity
    // 2 kNbMaxHalf dy then 2 kNbMaxHalf dx (visible to all after the first tile's barrier)
    [[maybe_unused]] KOHLER_LDS int8_t *foffs =
        reinterpret_cast<KOHLER_LDS int8_t *>(reinterpret_cast<KOHLER_LDS uint8_t *>(lds) + q.offs_off);
    if constexpr (FORM == FORM_MARG) {
        if (threadIdx.x < 8 * kNbMaxHalf) {
            const int par = (int)threadIdx.x / (4 * kNbMaxHalf), i = (int)threadIdx.x % (4 * kNbMaxHalf);
            foffs[threadIdx.x] = i < 2 * kNbMaxHalf ? q.fdy[par][i] : q.fdx[par][i - 2 * kNbMaxHalf];
        }
    }
    // tile t: first row r0, first column c0
    auto tile_at = [&](int64_t t, int64_t &r0, int &c0) {
        const int64_t ty = t / q.tiles_x;
        r0 = ty * TH;
        c0 = (int)(t - ty * q.tiles_x) * TW;
    };
    // 1. the tile's values. Unfiltered: rows r0 .. r0 + TH + R - 1 and columns c0 - R .. c0 + TW + R - 1
    //    into the tile (kNbOut outside the image). Filtered: one more row and column on every side
    //    into the raw tile, with coordinates clamped into the image (the filter's border rule), then
    //    the filter from LDS into the tile. Each image pixel is range-checked by the tile that owns it.
    const int st_rows = TH + R + 2 * F, st_cols = TC + 2 * F;
    StageRegs sr;
    // the staged region of tile t (its row stride in LDS is its width)
    auto region_of = [&](int64_t t) {
        int64_t r0;
        int c0;
        tile_at(t, r0, c0);
        const int own = (int)min<int64_t>(TH, H - r0);
        return F ? StageRegion{r0 - 1, c0 - R - 1, st_rows, st_cols, 1, own, R + 1}
                 : StageRegion{r0, c0 - R, st_rows, st_cols, 0, own, R};
    };
    auto load_tile = [&](int64_t t) { load_region<Pix>(im, region_of(t), sr); };
    if (g < q.tiles) load_tile(g);
    for (int64_t t = g; t < q.tiles; t += G, ++mine) {
        int64_t r0;
        int c0;
        tile_at(t, r0, c0);
        const int rows_left = (int)min<int64_t>(H - r0, (int64_t)1 << 30);  // image rows from r0 on
        const int above = r0 > kNbMaxRadius ? kNbMaxRadius : (int)r0;        // image rows above r0 in reach
        const int own = min(TH, rows_left);
        // every pixel of the tile has its whole neighbourhood inside the image (all R rows and columns
        // around the tile are image pixels): no pair or degree needs a test
        const bool interior = r0 >= R && TH + R <= rows_left && c0 >= R && c0 + TW + R <= W32;
        if (F) store_region<STAGE_RAW, CLAMP>(im, region_of(t), sr, raw, Mm1, vmax);
        else store_region<STAGE_MARK, CLAMP>(im, region_of(t), sr, tile, Mm1, vmax);
        __syncthreads();
        if (F) {
            for (int rx = (int)threadIdx.x; rx < TC; rx += TW) {
                const int xf = c0 - R + rx;
                const bool xout = xf < 0 || xf >= W32;
                const KOHLER_LDS uint16_t *s = raw + rx;
                auto hsum = [&](int i) {
                    return (uint32_t)s[i * (TC + 2)] + 2u * (uint32_t)s[i * (TC + 2) + 1] + (uint32_t)s[i * (TC + 2) + 2];
                };
                uint32_t h0 = hsum(0), h1 = hsum(1);
                for (int ry = 0; ry < TH + R; ++ry) {
                    const uint32_t h2 = hsum(ry + 2);
                    uint32_t v = (h0 + 2u * h1 + h2 + 8u) >> 4;
                    if constexpr (CLAMP) v = min(v, Mm1);
                    tile[ry * TC + rx] = (uint16_t)((xout || ry >= rows_left) ? kNbOut : v);
                    h0 = h1;
                    h1 = h2;
                }
            }
            __syncthreads();
        }
        // the next tile's loads are in flight while this tile's pairs are formed
        if (t + G < q.tiles) load_tile(t + G);
        // 2. the pairs of the tile's own pixels, one column per thread, rows in groups of four (their
        //    LDS reads in flight together); a row of parity par takes that parity's half offsets. An
        //    interior tile takes every pair and the whole degree without a test.
        const int x = c0 + (int)threadIdx.x;
        const int par0 = (int)(r0 & 1);
        const KOHLER_LDS uint16_t *col = tile + R + (int)threadIdx.x;
        auto pass = [&](auto in_tag) {
            constexpr bool IN = decltype(in_tag)::value;
            for (int ry = 0; ry < own; ry += 4) {
                uint32_t v[4];
                typename Acc::P pv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    v[k] = col[min(ry + k, own - 1) * TC];
                    pv[k] = Acc::prep(v[k]);
                }
                for (int a = 0; a < na_max; ++a) {
                    uint32_t w[4];
                    bool ok[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int pk = (par0 + k) & 1;  // ry is a multiple of 4
                        const int o = __builtin_amdgcn_readlane(offv, 16 * pk + a);
                        const int r = min(ry + k, own - 1);
                        // the row and the offset exist (uniform); then, off the interior, both pixels
                        // lie inside the image
                        ok[k] = ry + k < own && a < (pk ? na1 : na0);
                        // offsets past a parity's count are zero: the read stays on the tile
                        w[k] = col[r * TC + o];
                        if constexpr (!IN) ok[k] = ok[k] && max(v[k], w[k]) != kNbOut;
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if constexpr (IN) {
                            if (ok[k]) acc.pair(pv[k], Acc::prep(w[k]), true);
                        } else {
                            acc.pair(pv[k], Acc::prep(w[k]), ok[k]);
                        }
                    }
                }
                if constexpr (FORM == FORM_MARG) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int pk = (par0 + k) & 1;
                        const int nf = pk ? nf1 : nf0;
                        const int ryk = ry + k;
                        if constexpr (IN) {
                            if (ryk < own) acc.pixel(v[k], (uint32_t)nf, true);
                        } else {
                            // a pixel at least R rows and columns inside the image has the whole neighbourhood
                            uint32_t deg = (uint32_t)nf;
                            if (!(ryk >= R - above && ryk < rows_left - R && x >= R && x < W32 - R)) {
                                deg = 0;
                                const KOHLER_LDS int8_t *fo = foffs + pk * 4 * kNbMaxHalf;
                                for (int b = 0; b < nf; ++b) {
                                    const int ry1 = ryk + fo[b], x1 = x + fo[2 * kNbMaxHalf + b];
                                    deg += (ry1 >= -above && ry1 < rows_left && (uint32_t)x1 < (uint32_t)W32) ? 1u : 0u;
                                }
                            }
                            acc.pixel(v[k], deg, ryk < own && v[k] != kNbOut);
                        }
                    }
                }
            }
        };
        if (interior) pass(std::true_type{});
        else pass(std::false_type{});
        __syncthreads();  // before the next tile is staged over this one
    }
    phase_wave_stamp();
    flush_image<FORM, CLAMP>(p, lds, bs, im, vmax, mine, q.tiles);
}

template <typename Pix>
const void *pick_nbhd_form(int form, bool clamp) {
    if (form == FORM_TRI)
        return clamp ? reinterpret_cast<const void *>(nbhd_kernel<Pix, FORM_TRI, true>)
                     : reinterpret_cast<const void *>(nbhd_kernel<Pix, FORM_TRI, false>);
    return clamp ? reinterpret_cast<const void *>(nbhd_kernel<Pix, FORM_MARG, true>)
                 : reinterpret_cast<const void *>(nbhd_kernel<Pix, FORM_MARG, false>);
}

const void *pick_nbhd_kernel(int dtype, int form, int M) {
    return dtype == 1 ? pick_nbhd_form<uint8_t>(form, M < 256) : pick_nbhd_form<uint16_t>(form, true);
}

template <typename Pix, int NB, int K>
const void *pick_form(int form, bool clamp) {
    if (form == FORM_BAND)
        return clamp ? reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_BAND, true>)
                     : reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_BAND, false>);
    if (form == FORM_TRI)
        return clamp ? reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_TRI, true>)
                     : reinterpret_cast<const void *>(curve_kernel<Pix, NB, K, FORM_TRI, false>);
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

// hipFuncSetAttribute and the occupancy query cost host time on every call, so their results are
// kept per device and kernel (the occupancy per block size and LDS bytes too) in fixed tables: no
// heap allocation, and when a table is full the call is simply made again.
constexpr int kKernCache = 256;
struct KernCache {
    std::mutex mu;
    int n_attr = 0, n_occ = 0;
    struct Attr {
        int dev;
        const void *kern;
    } attr[kKernCache];
    struct Occ {
        int dev;
        const void *kern;
        int block;
        size_t lds;
        int n;
    } occ[kKernCache];
};
KernCache &kern_cache() {
    static KernCache c;
    return c;
}

hipError_t allow_large_lds(const void *kern) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    KernCache &c = kern_cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (int i = 0; i < c.n_attr; ++i)
            if (c.attr[i].dev == dev && c.attr[i].kern == kern) return hipSuccess;
    }
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLdsBytes);
    if (e == hipSuccess) {
        std::lock_guard<std::mutex> lk(c.mu);
        if (c.n_attr < kKernCache) c.attr[c.n_attr++] = {dev, kern};
    }
    return e;
}

// Workgroups of `kern` with `block` threads and `lds` bytes that fit on one compute unit (>= 1).
int occupancy(const void *kern, int block, size_t lds) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    KernCache &c = kern_cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        for (int i = 0; i < c.n_occ; ++i)
            if (c.occ[i].dev == dev && c.occ[i].kern == kern && c.occ[i].block == block && c.occ[i].lds == lds)
                return c.occ[i].n;
    }
    if (allow_large_lds(kern) != hipSuccess) return 1;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block, lds) != hipSuccess) return 1;
    n = n > 0 ? n : 1;
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.n_occ < kKernCache) c.occ[c.n_occ++] = {dev, kern, block, lds, n};
    return n;
}

}  // namespace

hipError_t curve_kernel_for(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block,
                            int copies, const void **func, size_t *lds) {
    *lds = lds_bytes(form, M, band, block, copies);
    *func = pick_kernel(dtype, nbhd, form, px_per_lane, M);
    return allow_large_lds(*func);
}

hipError_t launch_curve(const KParams &p, int dtype, int nbhd, int form, int px_per_lane, int block,
                        int grid, hipStream_t stream) {
    const size_t lds = lds_bytes(form, p.M, p.band, block, p.copies);
    const void *kern = pick_kernel(dtype, nbhd, form, px_per_lane, p.M);
    hipError_t e = allow_large_lds(kern);
    if (e != hipSuccess) return e;
    KParams arg = p;
    void *args[] = {&arg};
    e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

int max_block_for(int dtype, int nbhd, int form, int px_per_lane, int M) {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, pick_kernel(dtype, nbhd, form, px_per_lane, M)) != hipSuccess) return 0;
    return a.maxThreadsPerBlock;
}

int blocks_per_cu(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block, int copies) {
    return occupancy(pick_kernel(dtype, nbhd, form, px_per_lane, M), block, lds_bytes(form, M, band, block, copies));
}

size_t nbhd_lds_layout(NbParams &q, int form, int block) {
    // the tables (or the finishing step's arrays) first, then the value tile, then (pre-filter only)
    // the raw tile with one more row and column on every side, then the whole-neighbourhood offsets,
    // then the scratch. Tile rows: the most that fit, at most 16.
    const size_t table = lds_main_bytes(form, q.k.M, 1, block, 1);
    const size_t tile_off = (table + 15) & ~(size_t)15;
    const int R = q.radius, F = q.filter ? 1 : 0;
    const size_t room = kMaxLdsBytes - sizeof(BlockScratch) - 16;
    auto bytes_for = [&](int rows, size_t &raw_off, size_t &bs_off) {
        const size_t tile = (size_t)(rows + R) * (size_t)(block + 2 * R) * sizeof(uint16_t);
        raw_off = (tile_off + tile + 15) & ~(size_t)15;
        const size_t rawb = F ? (size_t)(rows + R + 2) * (size_t)(block + 2 * R + 2) * sizeof(uint16_t) : 0;
        q.offs_off = (uint32_t)((raw_off + rawb + 15) & ~(size_t)15);
        bs_off = (q.offs_off + 8 * kNbMaxHalf + 15) & ~(size_t)15;
        return bs_off;
    };
    int best = 16;
    size_t raw_off = 0, bs_off = 0;
    while (best > 1 && bytes_for(best, raw_off, bs_off) > room) --best;
    bytes_for(best, raw_off, bs_off);
    q.tile_rows = best;
    q.tile_off = (uint32_t)tile_off;
    q.raw_off = (uint32_t)raw_off;
    q.bs_off = (uint32_t)bs_off;
    return bs_off + sizeof(BlockScratch);
}

int nbhd_blocks_per_cu(int dtype, int form, int M, int block, size_t lds) {
    return occupancy(pick_nbhd_kernel(dtype, form, M), block, lds);
}

hipError_t launch_nbhd(const NbParams &q, int dtype, int form, int block, int grid, size_t lds,
                       hipStream_t stream) {
    const void *kern = pick_nbhd_kernel(dtype, form, q.k.M);
    hipError_t e = allow_large_lds(kern);
    if (e != hipSuccess) return e;
    NbParams arg = q;
    void *args[] = {&arg};
    e = hipLaunchKernel(kern, dim3(grid), dim3(block), args, lds, stream);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace kohler

#ifdef KOHLER_PHASE_CLOCK
// Measurement build only: copy (and optionally clear) the phase timestamps of the last launches.
// `slots` receives kPhaseMaxWG * kPhaseSlots words, `waves` kPhaseMaxWG * kPhaseWaves words.
extern "C" __attribute__((visibility("default"))) int kohler_phase_clock_read(unsigned long long *slots,
                                                                               unsigned long long *waves,
                                                                               int clear) {
    using namespace kohler;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && slots)
        e = hipMemcpyFromSymbol(slots, HIP_SYMBOL(g_phase), sizeof(g_phase), 0, hipMemcpyDeviceToHost);
    if (e == hipSuccess && waves)
        e = hipMemcpyFromSymbol(waves, HIP_SYMBOL(g_phase_wave), sizeof(g_phase_wave), 0, hipMemcpyDeviceToHost);
    if (e == hipSuccess && clear) {
        void *a = nullptr, *b = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(g_phase));
        if (e == hipSuccess) e = hipGetSymbolAddress(&b, HIP_SYMBOL(g_phase_wave));
        if (e == hipSuccess) e = hipMemset(a, 0, sizeof(g_phase));
        if (e == hipSuccess) e = hipMemset(b, 0, sizeof(g_phase_wave));
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    return e == hipSuccess ? 0 : -5;
}
#endif
