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
};

// Kernel arguments. Outputs and scratch are image-major: image i uses acc + i*2*M, sum + i*M,
// thr + i*cap, n_thr + i, and so on.
struct KParams {
    const KImage *imgs;   // device table, used when n > 1
    KImage img0;          // inline descriptor, used when n == 1
    int32_t n, M, band, cap;
    int64_t total_units;
    int64_t *acc;         // [n][2M] int64: first-difference array of #B(t), then second-difference
                          // array of the contrast sums; all zero between launches
    unsigned long long *done;  // [n] units completed in the current launch; zero between launches
    uint32_t *rflag;      // [n] set when a pixel >= M was seen; zero between launches
    int64_t *sum;
    int64_t *count;
    double *C;
    int32_t *thr;
    int32_t *n_thr;
    int32_t *t0;
    int32_t *status;
};

enum Form { FORM_BAND = 1, FORM_MARG = 2 };

// Largest grey-level range that fits each form's LDS tables.
constexpr int kMaxMBand = 256;
constexpr int kMaxMMarg = 10200;
constexpr int kMaxBandRows = 64;
constexpr size_t kMaxLdsBytes = 160 * 1024;

// LDS bytes a launch needs for (form, M, band).
size_t lds_bytes(int form, int M, int band);

// Workgroups of this launch family that fit on one compute unit at once.
int blocks_per_cu(int dtype, int nbhd, int form, int px_per_lane, int M, int band, int block);

// Launch the curve kernel. Returns hipSuccess or the launch error.
hipError_t launch_curve(const KParams &p, int dtype, int nbhd, int form, int px_per_lane, int block,
                        int grid, hipStream_t stream);

}  // namespace kohler
