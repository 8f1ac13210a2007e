// Internal interface between the C-ABI layer (kohler_api.cpp) and the gfx950 kernels
// (kohler_kernels.hip). Not installed; the public interface is include/kohler.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kohler {

// One image of a launch. Work is cut into "units": one unit is one row of one vertical strip of
// 64 * px_per_lane columns, so an image has nunits = nstrips * H units, numbered strip-major
// (unit = strip * H + row). ustart is the first unit of this image in the launch's unit space.
struct KImage {
    const void *ptr;
    int64_t H, W, pitch;  // pitch in elements
    int64_t ustart;
    int64_t nunits;
    int32_t nstrips;
    int32_t vec_ok;       // 1 when base and pitch allow aligned vector loads of px_per_lane pixels
    int32_t out;          // index of this image's outputs and scratch (see KParams)
    int32_t pad;
};

// Kernel arguments. Outputs and scratch are indexed by the image's `out` field o: the image uses the
// accumulators at acc + o*acc_stride, done[o] and rflag[o], and writes sum + o*ostride,
// count + o*ostride, C + o*ostride (M values each), thr + o*istride (cap values), n_thr + o*istride,
// t0 + o*istride and status + o*istride. A batch call numbers its images 0..n-1 with ostride = M,
// istride = 1 for the scalars and cap for thr (thr_stride); the server gives each image the index
// of the slot that holds it and lays a slot's outputs out as one record.
struct KParams {
    const KImage *imgs;   // device table, used when n > 1
    KImage img0;          // inline descriptor, used when n == 1
    int32_t n, M, band, cap;
    int32_t packed_acc;   // 1: acc holds E * 2^32 + D1 in one word per level (images small enough)
    int32_t nrep;         // accumulator replicas per image; workgroup b adds into replica b % nrep
    int64_t rep_stride;   // int64 words between replicas (>= 2M)
    int64_t acc_stride;   // int64 words between the accumulators of two output indices (>= nrep*rep_stride)
    int64_t total_units;
    int64_t *acc;         // per output index, nrep replicas of rep_stride int64 words: the
                          // first-difference array of #B(t) then the second-difference array of the
                          // contrast sums (or both packed in the first M words); zero between launches
    unsigned long long *done;  // per output index: units completed in the current launch; zero between launches
    int32_t dyn;          // 1: one image, chunks dealt round-robin to the workgroups
    int32_t copies;       // banded form: copies of the joint table per workgroup (lane l uses copy l % copies)
    uint32_t *rflag;      // per output index: set when a pixel >= M was seen; zero between launches
    int64_t ostride;      // elements between the sum/count/C arrays of two output indices
    int64_t istride;      // elements between the n_thr/t0/status entries of two output indices
    int64_t thr_stride;   // elements between the thr arrays of two output indices
    int64_t *sum;
    int64_t *count;
    double *C;
    int32_t *thr;
    int32_t *n_thr;
    int32_t *t0;
    int32_t *status;
};

enum Form { FORM_BAND = 1, FORM_MARG = 2, FORM_TRI = 3 };

// Accumulator replicas: spreading the workgroups' global atomics over several copies keeps the
// number of workgroups that contend for one word small.
constexpr int kMaxReplicas = 16;
inline int64_t replica_stride(int M) { return ((int64_t)2 * M + 511) / 512 * 512; }

// Largest grey-level range that fits each form's LDS tables.
constexpr int kMaxMBand = 256;
constexpr int kMaxMMarg = 10200;
constexpr int kMaxBandRows = 64;
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Workgroup scratch for the block-wide scans and reductions; lives at the end of dynamic LDS so that
// the histogram table starts at LDS address 0.
struct BlockScratch {
    int64_t scan[16];
    int64_t red_s[16];
    int64_t red_k[16];
    int32_t red_t[16];
    int32_t last;
    uint32_t next;   // next unclaimed chunk of the workgroup's current segment
    int32_t pad[2];
};

// Words between two rows of the banded table (at least 257: a row holds 256 low values, and the
// word after them must stay zero, see merge_band). The stride sets which LDS bank a counter (d, lo)
// falls in, (d * stride + lo) mod banks: with 257 the bank is hi mod banks, which neighbouring pixels
// of a smooth image share; a stride of 256 + 16 spreads the gaps over the banks as well.
#ifndef KOHLER_ROW_STRIDE
#define KOHLER_ROW_STRIDE 272
#endif
constexpr int kRowStride = KOHLER_ROW_STRIDE;
static_assert(kRowStride >= 257, "a row of the banded table needs 256 counters and one zero word");

// Copies of the banded table a workgroup may keep (lanes spread over them, so fewer lanes of one
// LDS instruction add to the same counter).
constexpr int kMaxBandCopies = 4;

// LDS bytes before the BlockScratch: the histogram tables, or the finalize step's arrays, whichever
// is larger; 16-byte aligned. Finalize for M <= 256 needs 8 KiB (the curve and per-wave masks); for
// larger M, two int64 arrays of block + 1 entries and one byte per grey level.
// Finishing step for M > 256: M flag bytes (within the first 16 (block + 1) + M bytes), then (from
// this byte offset) the replica sums of the M levels, one uint64 each, in ceil(M / block) rows of
// block words (thread j's levels in column j).
__host__ __device__ inline size_t fin_gather_offset(int M, int block) {
    return (16 * ((size_t)block + 1) + (size_t)M + 15) & ~(size_t)15;
}

__host__ __device__ inline size_t lds_main_bytes(int form, int M, int band, int block, int copies) {
    // banded form: `copies` tables of band + 2 rows, then the hmax and hsum tables of the gaps beyond
    // the band (768 words); triangular form: M (M + 1) / 2 counters, 64 invalid-pair words, then
    // hmin, hmax (M each) and hsum (2M, one spare)
    const size_t words = (form == FORM_BAND)  ? (size_t)copies * ((size_t)band + 2) * kRowStride + 768
                         : (form == FORM_TRI) ? (size_t)M * (M + 1) / 2 + 64 + 4 * (size_t)M
                                              : 4 * (size_t)M * (size_t)copies;
    const size_t table = (words * 4 + 15) & ~(size_t)15;
    const size_t fin = M <= 256 ? (size_t)8192
                                : fin_gather_offset(M, block) + 8 * (((size_t)M + block - 1) / block) * (size_t)block;
    return table > fin ? table : fin;
}

// LDS bytes a launch needs for (form, M, band, threads per workgroup, table copies).
inline size_t lds_bytes(int form, int M, int band, int block, int copies) {
    return lds_main_bytes(form, M, band, block, copies) + sizeof(BlockScratch);
}

// Largest workgroup (threads) the kernel instance of a launch family was compiled for (0 on error).
int max_block_for(int dtype, int nbhd, int form, int px_per_lane, int M);

// Workgroups of this launch family that fit on one compute unit at once.
int blocks_per_cu(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block, int copies);

// The kernel instance of a launch family and the dynamic LDS bytes it needs (for graph kernel
// nodes); allows the kernel to use that much LDS.
hipError_t curve_kernel_for(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block,
                            int copies, const void **func, size_t *lds);

// ------------------------------------------------------------------------------------------------
// Other neighbourhoods and the pre-filter (one image per launch, nbhd_kernel): the pairs of a
// symmetric structuring element given by its half, or of the hexagonal grid (half offsets that
// depend on the row's parity), over tiles of tile_rows x blockDim pixels staged in LDS as 16-bit
// values (raw, or through the 3x3 binomial pre-filter). Joint (triangular) table for M <= 256,
// marginal histograms above.

constexpr int kNbMaxHalf = 16;    // half offsets per row parity
constexpr int kNbMaxRadius = 7;   // largest |dx| and dy of a half offset
constexpr int kNbBlock = 512;     // threads per workgroup = tile columns
constexpr int kNbMaxM = 8192;     // marginal tables plus the tile fit the LDS

struct NbParams {
    KParams k;                    // the image, scratch and outputs as for a single-image curve launch
    int32_t nhalf[2];             // half offsets of even and odd rows
    int32_t nfull[2];             // whole-neighbourhood offsets of even and odd rows (pixel degrees)
    int8_t hdy[2][kNbMaxHalf], hdx[2][kNbMaxHalf];
    int8_t fdy[2][2 * kNbMaxHalf], fdx[2][2 * kNbMaxHalf];
    int32_t radius;               // largest |dx| and dy over the half offsets
    int32_t filter;               // 1: 3x3 binomial pre-filter, rounded half up, replicated borders
    int32_t tile_rows;            // image rows per tile
    uint32_t tile_off;            // LDS byte offset of the value tile
    uint32_t bs_off;              // LDS byte offset of the workgroup scratch
    uint32_t raw_off;             // LDS byte offset of the unfiltered tile (pre-filter only)
    uint32_t offs_off;            // LDS byte offset of the copy of fdy, fdx (8 kNbMaxHalf bytes)
    int32_t pad;
    int64_t tiles_x, tiles;       // tiles per band of tile_rows rows, and in all
};

// LDS layout of an nbhd_kernel launch: fills tile_rows, tile_off, raw_off, offs_off and bs_off and returns the
// bytes (radius, filter and k.M set).
size_t nbhd_lds_layout(NbParams &q, int form, int block);
// Workgroups of an nbhd_kernel instance that fit on one compute unit.
int nbhd_blocks_per_cu(int dtype, int form, int M, int block, size_t lds);
// Launch nbhd_kernel (every field of q set). Returns hipSuccess or the launch error.
hipError_t launch_nbhd(const NbParams &q, int dtype, int form, int block, int grid, size_t lds,
                       hipStream_t stream);

// ------------------------------------------------------------------------------------------------
// Two-class segmentation at a device-resident t0 (the serving loop's video mode, eq (4)): label 1
// where f > t0, else 0; every pixel 0 when t0 < 0 (the curve is identically zero: one class).

struct LabelJob {
    const void *img;       // H rows of `pitch` elements of the launch's dtype (device)
    uint8_t *labels;       // H rows of `lpitch` bytes (device)
    const int32_t *t0;     // device
    int64_t H, W, pitch, lpitch;
};
constexpr int kMaxLabelJobs = 16;
struct LabelJobs {
    LabelJob job[kMaxLabelJobs];
    int32_t n, dtype;
};
// One launch labelling js.n images (1..kMaxLabelJobs). Returns hipSuccess or the launch error.
hipError_t launch_label_t0(const LabelJobs &js, hipStream_t stream);

// Launch the curve kernel (p.band and p.copies already set). Returns hipSuccess or the launch error.
hipError_t launch_curve(const KParams &p, int dtype, int nbhd, int form, int px_per_lane, int block,
                        int grid, hipStream_t stream);

}  // namespace kohler
