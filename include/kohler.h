/*
 * kohler.h — C ABI of the MI355X (gfx950) implementation of Köhler's contrast-thresholding curve.
 *
 * Reference: G. Noyel, "Speeding up the Köhler's method of contrast thresholding",
 * arXiv 1707.05062.
 *
 * What is computed (Sec. 2.1, eqs (1)-(4)). An image f has H rows and W columns of integer grey
 * levels in [0, M). For each integer threshold t in [0, M), the boundary B(t) is the set of ordered
 * pairs (x0, x1) of neighbouring pixels with f(x0) <= t < f(x1) (eq (1)); each pair has the contrast
 * min(f(x1) - t, t - f(x0)) (eq (2)). The library returns, for every t,
 *     sum[t]   = sum of the contrasts over B(t)              (exact, int64)
 *     count[t] = #B(t)                                       (exact, int64)
 *     C[t]     = sum[t] / count[t], or 0 when B(t) is empty  (eq (3); one IEEE binary64 division)
 * the local maxima of C in ascending order (the multiple thresholds of Sec. 2.1), and the optimal
 * threshold t0 of eq (4).
 *
 * Neighbourhoods: nbhd = 4 (the 4-neighbourhood N4 used throughout the paper) or nbhd = 8 (the
 * 8-neighbourhood it mentions as an alternative in Sec. 2). Pairs exist only between two pixels of
 * the image: there is no wrap-around and no padding.
 *
 * Local maxima: a maximal run [a, b] of equal positive C values is a local maximum when its outer
 * neighbours are strictly smaller (a = 0 or C(a-1) < C(a); b = M-1 or C(b+1) < C(b)); it is reported
 * at a. t0 is the smallest t attaining max C, or -1 when C is identically zero. Curve values are
 * compared exactly (as rationals sum/count), never as rounded doubles.
 *
 * Conventions for every entry point:
 *   - Images are row-major; pitch is the distance between row starts in ELEMENTS (pitch >= W).
 *     dtype KOHLER_U8 reads uint8_t pixels, KOHLER_U16 reads uint16_t pixels.
 *   - Valid sizes: H >= 1, 1 <= W <= 2^30, H * W <= 2^40; 1 <= M <= 256 for KOHLER_U8 and
 *     1 <= M <= KOHLER_MAX_M_U16 for KOHLER_U16; nbhd in {4, 8}; thr_capacity >= 0.
 *   - Arguments are checked before any device work. A bad argument returns KOHLER_E_ARG and leaves
 *     every output untouched.
 *   - A pixel value >= M is detected on the device; the call then reports KOHLER_E_RANGE and the
 *     outputs are unspecified (no memory outside the documented buffers is touched).
 *   - More local maxima than thr_capacity: the first thr_capacity are written, *n_thresholds gets
 *     the full number, and the status is KOHLER_E_CAPACITY (sum, count, C and t0 are still valid).
 *   - The caller owns every input and output buffer. A context owns its device scratch; nothing is
 *     allocated per call once a context has seen the largest shape it will serve, except where an
 *     entry point says otherwise.
 *   - One context runs one call at a time: calls that share a context must be ordered on one
 *     stream (or synchronised by the caller). Separate contexts are independent.
 */
#ifndef KOHLER_H
#define KOHLER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kohler_ctx kohler_ctx;
typedef struct ihipStream_t *kohler_stream_t; /* a hipStream_t; NULL means the null stream */

enum kohler_status {
    KOHLER_OK = 0,
    KOHLER_E_ARG = -1,      /* invalid argument (checked on the host before any device work) */
    KOHLER_E_RANGE = -2,    /* some pixel is >= M */
    KOHLER_E_CAPACITY = -3, /* more local maxima than thr_capacity */
    KOHLER_E_NOMEM = -4,    /* device or pinned host allocation failed */
    KOHLER_E_DEVICE = -5,   /* a HIP runtime call failed */
    KOHLER_E_BUSY = -6      /* admission refused (serving: HBM budget or queue full) */
};

enum kohler_dtype { KOHLER_U8 = 1, KOHLER_U16 = 2 };

#define KOHLER_MAX_M_U16 10200

/*
 * Create a context on HIP device `device`. It allocates the scratch for single-image calls up to
 * the largest M, a pinned staging area for the synchronous entry point, and a stream of its own.
 * Returns KOHLER_OK, KOHLER_E_ARG (out == NULL or no such device), KOHLER_E_NOMEM or
 * KOHLER_E_DEVICE. On failure *out is set to NULL.
 */
int kohler_create(kohler_ctx **out, int device);

/* Destroy a context after waiting for its work. NULL is a no-op. */
void kohler_destroy(kohler_ctx *ctx);

/* Static string describing a status code (never NULL). */
const char *kohler_strerror(int status);

/*
 * Synchronous curve of one image (Sec. 2.1, eqs (1)-(4); result equal to Algorithm 1 of Sec. 3.1).
 *   img          device or host pointer to H rows of `pitch` elements of `dtype`; a host image is
 *                copied to the device through the context's staging buffer first.
 *   sum, count   HOST arrays of M int64 (required).
 *   C            HOST array of M doubles (required).
 *   thresholds   HOST array of thr_capacity int32 (may be NULL when thr_capacity == 0).
 *   n_thresholds, t0   HOST int32 (required).
 * Returns when the results are in host memory. Status as described above.
 */
int kohler_curve(kohler_ctx *ctx, const void *img, int dtype, int64_t H, int64_t W, int64_t pitch,
                 int32_t M, int32_t nbhd, int64_t *sum, int64_t *count, double *C,
                 int32_t *thresholds, int32_t thr_capacity, int32_t *n_thresholds, int32_t *t0);

/*
 * Stream-ordered curve of one image. Every pointer is DEVICE memory: d_img as in kohler_curve;
 * d_sum, d_count (M int64), d_C (M doubles), d_thr (thr_capacity int32, may be NULL when the
 * capacity is 0), d_n_thr, d_t0, d_status (one int32 each). The device writes the call's status
 * (KOHLER_OK, KOHLER_E_RANGE or KOHLER_E_CAPACITY) to *d_status. The return value covers only the
 * host-side checks and the launch (KOHLER_OK, KOHLER_E_ARG, KOHLER_E_DEVICE). One kernel launch,
 * no host synchronisation, no allocation.
 */
int kohler_curve_async(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W,
                       int64_t pitch, int32_t M, int32_t nbhd, int64_t *d_sum, int64_t *d_count,
                       double *d_C, int32_t *d_thr, int32_t thr_capacity, int32_t *d_n_thr,
                       int32_t *d_t0, int32_t *d_status, kohler_stream_t stream);

/*
 * Stream-ordered curves of n images of possibly different shapes in ONE persistent launch
 * (images are independent: no pair crosses two images). Host arrays d_imgs[n] (device pointers),
 * H[n], W[n], pitch[n] describe the images; all share dtype, M and nbhd. Outputs are DEVICE
 * arrays laid out image-major: d_sum[n*M], d_count[n*M], d_C[n*M], d_thr[n*thr_capacity],
 * d_n_thr[n], d_t0[n], d_status[n]. The context grows its batch scratch to the largest n seen
 * (the only allocation, made before the launch); the per-image descriptor table is copied to the
 * device on `stream`. Returns as kohler_curve_async.
 */
int kohler_curve_batch(kohler_ctx *ctx, int32_t n, const void *const *d_imgs, const int64_t *H,
                       const int64_t *W, const int64_t *pitch, int dtype, int32_t M, int32_t nbhd,
                       int64_t *d_sum, int64_t *d_count, double *d_C, int32_t *d_thr,
                       int32_t thr_capacity, int32_t *d_n_thr, int32_t *d_t0, int32_t *d_status,
                       kohler_stream_t stream);

/*
 * Launch plan control (the autotuner's knobs). A plan fixes, for one (dtype, M, nbhd) family:
 *   form        0 = automatic, 1 = banded joint histogram (M <= 256), 2 = marginal histograms
 *   band        number of gap rows of the banded table (2..64; form 1 only)
 *   block       threads per workgroup (256 or 512)
 *   grid        workgroups per launch (0 = automatic: enough to fill every compute unit)
 *   px_per_lane pixels each lane loads per row (4 or 8 for KOHLER_U8, 4 for KOHLER_U16)
 * kohler_set_plan stores a plan in the context for later calls (KOHLER_E_ARG if it is invalid);
 * kohler_get_plan reports the plan a call with these parameters would use.
 */
typedef struct kohler_plan {
    int32_t form;
    int32_t band;
    int32_t block;
    int32_t grid;
    int32_t px_per_lane;
} kohler_plan;

int kohler_set_plan(kohler_ctx *ctx, int dtype, int32_t M, int32_t nbhd, const kohler_plan *plan);
int kohler_get_plan(kohler_ctx *ctx, int dtype, int64_t H, int64_t W, int32_t M, int32_t nbhd,
                    kohler_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* KOHLER_H */
