// Host-side internals shared by the C-ABI sources (kohler_api.cpp, kohler_server.cpp): the context
// object and the argument, plan and descriptor helpers. Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>

#include "kohler.h"
#include "kohler_impl.h"

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
    kohler::KImage *d_table = nullptr;
    kohler::KImage *h_table = nullptr;  // pinned
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

    // class statistics: grey-level histogram (kMaxM + 1 words), allocated on first use, zero between calls
    unsigned long long *level_hist = nullptr;

    std::map<std::tuple<int, int, int>, kohler_plan> plans;
    std::mutex mu;
};

namespace kohler {

constexpr int kMaxM = std::max(kMaxMBand, kMaxMMarg);

// Status code of a HIP error.
int pick_status(hipError_t e);
// Host-side check of an image shape and its family (see the size rules in include/kohler.h).
bool valid_shape(int dtype, int64_t H, int64_t W, int64_t pitch, int32_t M, int32_t nbhd);
bool valid_plan(const kohler_plan &pl, int dtype, int32_t M);
kohler_plan default_plan(int dtype, int32_t M);
// Plan for a call over `total_units` units: the stored plan of the family, else the default, with
// grid and replicas filled in.
kohler_plan resolve_plan(kohler_ctx *ctx, int dtype, int32_t M, int32_t nbhd, int64_t total_units);
int replicas_for(int grid);
// Fewest workgroups for a launch over `units` tile rows so that no 32-bit LDS counter overflows.
int min_grid_for(const kohler_plan &pl, int32_t nbhd, int64_t units);
// Whether one int64 word per grey level can hold both difference arrays of this image.
bool packable(int64_t H, int64_t W, int32_t nbhd);
int64_t strips_of(int64_t W, int px_per_lane);
// Kernel descriptor of one image (out index 0).
KImage describe(const void *ptr, int dtype, int64_t H, int64_t W, int64_t pitch, int px_per_lane,
                int64_t ustart);

}  // namespace kohler
