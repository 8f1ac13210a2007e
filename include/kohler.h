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
 *     outputs are unspecified (no memory outside the documented buffers is touched). This is the
 *     rule of every entry point that computes a curve. The consumers of thresholds already
 *     computed (kohler_segment, kohler_class_stats, kohler_mean_image) follow a different rule on
 *     purpose: they must give every pixel a class and have no device status word, so a value >= M
 *     is placed in the top class (it lies above every threshold), counted at the value M. Chained
 *     after a curve call on the same image, they inherit that call's KOHLER_E_RANGE, which the
 *     caller checks before trusting either.
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
    KOHLER_E_BUSY = -6,     /* admission refused (serving: HBM budget or queue full) */
    KOHLER_E_CANCELED = -7  /* serving: the request was cancelled before it ran */
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
 *                copied to the device through the context's staging buffer first. The call works
 *                on the context's own stream, which does not wait for any other stream: a device
 *                image must be complete (every write to it finished) when the call is made.
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
 * Other neighbourhoods and a pre-filter. Sec. 2.1 allows the 6-neighbourhood besides N4 and N8,
 * and the argument of Sec. 3.2 (eqs (7)-(9): every unordered pair counted once through a half
 * neighbourhood) holds for any symmetric structuring element A (a in A <=> -a in A) with a half A*
 * holding one offset of each pair {a, -a}. Sec. 5 suggests combining the method with a previous
 * low-pass filter; the one offered is a reading, the paper names none.
 *   kind KOHLER_NBHD_OFFSETS  A = A* u -A*, A* given as n_half (dy, dx) offsets (1..16, each
 *                             |dy|, |dx| <= 7, not (0, 0); an offset and its negation are the same
 *                             pairs and may appear only once), the same at every pixel;
 *   kind KOHLER_NBHD_HEX6     the 6-neighbourhood of a hexagonal grid stored on the H x W raster
 *                             with the odd rows shifted right by half a pixel: a pixel of an even
 *                             row y pairs with (y, x +- 1), (y +- 1, x - 1), (y +- 1, x); of an odd
 *                             row with (y, x +- 1), (y +- 1, x), (y +- 1, x + 1).
 *   prefilter 1: the curve of g = floor((sum of w f + 8) / 16) with the 3x3 binomial weights
 *             w = [1 2 1; 2 4 2; 1 2 1] and replicated borders (coordinates outside the image
 *             replaced by the nearest pixel) instead of f; g is computed on the fly, never stored.
 * Pairs exist only between pixels of the image. Stream-ordered as kohler_curve_async, with the same
 * device outputs and status values (a pixel >= M is a range error whether or not the filter is on);
 * sizes as there, with M <= 8192. Returns KOHLER_OK, KOHLER_E_ARG (checked on the host, also a bad
 * neighbourhood) or a launch error.
 */
enum kohler_nbhd_kind { KOHLER_NBHD_OFFSETS = 1, KOHLER_NBHD_HEX6 = 2 };
#define KOHLER_NBHD_MAX_HALF 16

typedef struct kohler_nbhd {
    int32_t kind;
    int32_t n_half;
    int32_t half_dy[KOHLER_NBHD_MAX_HALF];
    int32_t half_dx[KOHLER_NBHD_MAX_HALF];
} kohler_nbhd;

int kohler_curve_nbhd_async(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                            int32_t M, const kohler_nbhd *nbhd, int32_t prefilter, int64_t *d_sum,
                            int64_t *d_count, double *d_C, int32_t *d_thr, int32_t thr_capacity,
                            int32_t *d_n_thr, int32_t *d_t0, int32_t *d_status, kohler_stream_t stream);

/*
 * Launch plan control (the autotuner's knobs). A plan fixes, for one (dtype, M, nbhd) family:
 *   form        0 = automatic, 1 = banded joint histogram (M <= 256), 2 = marginal histograms,
 *               3 = triangular joint histogram of (lo, hi) (M <= 256)
 *   band        number of gap rows of the banded table (1..64; form 1 only)
 *   block       threads per workgroup (256, 512 or 1024)
 *   grid        workgroups per launch (0 = automatic: enough to fill every compute unit)
 *   px_per_lane pixels each lane loads per row (4 or 8 for KOHLER_U8, 4 for KOHLER_U16); a tile is
 *               one row of a strip of 64 * px_per_lane columns
 *   replicas    merge schedule: copies of the per-image device accumulators that the workgroups'
 *               partial histograms are added into (1..16; 0 = automatic, about one per 32
 *               workgroups); the finishing workgroup sums the copies
 *   copies      LDS privatisation width: copies of the tables each workgroup keeps, interleaved
 *               word by word, lane l of a wave adding to copy l % copies (banded form 1, 2 or 4;
 *               marginal form 1 or 2, as the LDS allows: 4 M words per copy; triangular form 1;
 *               0 = automatic: 2 for the banded form, else 1)
 *   acc_split   layout of the device accumulators: 0 = automatic (one int64 word per grey level
 *               holding E * 2^32 + D1 while the image, or every image of a batched launch, has
 *               fewer than 2^30 neighbour pairs, else two words), 1 = always two words (D1 and E
 *               apart: the layout very large images need, selectable for any image)
 * The grid is raised where needed so that no workgroup's 32-bit LDS counter can overflow: at least
 * ceil(w * 64 * px_per_lane * units / 2^31) workgroups for a launch over `units` tile rows, with w = 2
 * (nbhd 4) or 4 (nbhd 8) pairs per pixel, 8 for the marginal form.
 * kohler_set_plan stores a plan in the context for later calls (KOHLER_E_ARG if it is invalid);
 * kohler_get_plan reports the plan a call with these parameters would use.
 */
typedef struct kohler_plan {
    int32_t form;
    int32_t band;
    int32_t block;
    int32_t grid;
    int32_t px_per_lane;
    int32_t replicas;
    int32_t copies;
    int32_t acc_split;
} kohler_plan;

int kohler_set_plan(kohler_ctx *ctx, int dtype, int32_t M, int32_t nbhd, const kohler_plan *plan);
int kohler_get_plan(kohler_ctx *ctx, int dtype, int64_t H, int64_t W, int32_t M, int32_t nbhd,
                    kohler_plan *plan);

/* int64 words of accumulator scratch that kohler_curve_noalloc keeps per GPU (512 KiB). */
#define KOHLER_NOALLOC_SCRATCH_WORDS 65536

/*
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. The same computation and arguments as kohler_curve_async,
 * on the current HIP device, without a context: the kernel's scratch (accumulator replicas, ticket,
 * range flag) is a device array of the library, one per GPU, held until the process ends, and the
 * call makes no device or host allocation.
 *   plan     a launch plan as kohler_set_plan takes it (grid 0 = automatic), or NULL for the
 *            default plan; the replicas are limited to what the scratch holds
 *            (KOHLER_NOALLOC_SCRATCH_WORDS / the replica size, at least 3 for the largest M)
 * The first call on a device looks up and zeroes that device's array; every launch leaves it zeroed.
 * Calls on one GPU share the array: calls that overlap on the device race, so order them on one
 * stream. Returns KOHLER_OK, KOHLER_E_ARG (checked on the host; also an invalid plan) or
 * KOHLER_E_DEVICE; the device writes the status as for kohler_curve_async.
 */
int kohler_curve_noalloc(const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch, int32_t M,
                         int32_t nbhd, int64_t *d_sum, int64_t *d_count, double *d_C, int32_t *d_thr,
                         int32_t thr_capacity, int32_t *d_n_thr, int32_t *d_t0, int32_t *d_status,
                         const kohler_plan *plan, kohler_stream_t stream);

/*
 * Autotuner. Times candidate plans for the (dtype, M, nbhd) family on a representative workload
 * and stores the fastest in the context, as kohler_set_plan would. The workload is described as in
 * kohler_curve_batch (n device images; n == 1 tunes the single-image launch, n > 1 the batched
 * one). The search is a coordinate descent, two passes over the knobs in the order tile shape
 * (form and band), table copies, px_per_lane, block, grid (automatic or 1..4 workgroups per compute
 * unit) and replicas, starting from the default plan, then a joint sweep of band (banded form),
 * px_per_lane, grid and replicas (1, 2, 4, 8) around the result; each
 * candidate gets two warm-up launches and `reps` timed ones (0 means 5) on the context's stream,
 * and its median time counts. The device images must be complete when the call is made (the
 * context's stream does not wait for the caller's streams).
 *   best     out: the chosen plan (grid and replicas may be 0 = automatic)
 *   best_us  out (may be NULL): its median launch time in microseconds
 * It allocates and frees temporary device outputs and synchronises the context's stream, so it
 * belongs to set-up, not to a serving loop. Returns KOHLER_OK, KOHLER_E_ARG (bad workload), or a
 * launch/device error, in which case the context's previous plan for the family is restored.
 */
int kohler_autotune(kohler_ctx *ctx, int32_t n, const void *const *d_imgs, const int64_t *H,
                    const int64_t *W, const int64_t *pitch, int dtype, int32_t M, int32_t nbhd,
                    int32_t reps, kohler_plan *best, double *best_us);

/*
 * Segmentation by the thresholds (Sec. 2.1): the lower set of a threshold t is {f <= t} (eq (1)), so
 * ascending thresholds t_1 < ... < t_k cut the grey levels into k + 1 classes, and the pixel of value
 * f gets the label #{i : t_i < f} (0 .. k). Stream-ordered; every pointer is DEVICE memory:
 *   d_img, dtype, H, W, pitch, M   the image as for kohler_curve (values >= M take label k)
 *   d_thr            thresholds, strictly ascending in [0, M) (as kohler_curve_async writes them;
 *                    otherwise the labels are unspecified), at least min(*d_n_thr, thr_capacity)
 *   d_n_thr          one int32: how many thresholds there are (a count above thr_capacity, as a
 *                    capacity-truncated curve call reports it, uses the first thr_capacity)
 *   thr_capacity     0 .. M (host value)
 *   d_labels         H rows of label_pitch elements (label_pitch >= W) of label_dtype: KOHLER_U8
 *                    (needs thr_capacity <= 255) or KOHLER_U16
 * Each pixel is read once and each label written once (one kernel launch, no allocation, no host
 * synchronisation). Returns KOHLER_OK, KOHLER_E_ARG (checked on the host) or KOHLER_E_DEVICE.
 */
int kohler_segment(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                   int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                   void *d_labels, int label_dtype, int64_t label_pitch, kohler_stream_t stream);

/* Largest thr_capacity kohler_class_stats takes (its per-class sums are kept on chip). */
#define KOHLER_MAX_CLASS_THRESHOLDS 8000

/*
 * Class statistics of the segmentation by the thresholds (Sec. 2.1, where each class of Fig. 1 is
 * shown at the mean value of its pixels). Class j holds the pixels with label j as kohler_segment
 * gives it; a value of M or more counts in class k with the value M. Stream-ordered; every pointer is
 * DEVICE memory; image and thresholds as for kohler_segment, with thr_capacity <=
 * KOHLER_MAX_CLASS_THRESHOLDS.
 *   d_count, d_sum   int64[thr_capacity + 1]: pixels and sum of their values per class
 *   d_mean           double[thr_capacity + 1]: sum / count, one correctly rounded division, 0.0 for
 *                    an empty class
 * Entries past the n + 1 classes in use are 0. One kernel launch: a grey-level histogram (each
 * pixel read once) into a context scratch array, which the workgroup that finishes last folds into
 * the classes and clears; calls on one context must not overlap on the device (they share that
 * array).
 * Allocates the scratch on the first call. Returns KOHLER_OK, KOHLER_E_ARG, KOHLER_E_NOMEM or
 * KOHLER_E_DEVICE.
 */
int kohler_class_stats(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                       int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                       int64_t *d_count, int64_t *d_sum, double *d_mean, kohler_stream_t stream);

/*
 * The class-mean image (Sec. 2.1: the image simplified to one grey level per class, each class at
 * the mean value of its pixels): every pixel replaced by the mean of its class, rounded to the
 * nearest integer with ties to even, in the image's own type. Stream-ordered, DEVICE pointers:
 *   d_img .. thr_capacity   as for kohler_segment
 *   d_mean           double[thr_capacity + 1] class means (kohler_class_stats' d_mean); a value of
 *                    M or more takes class n's mean
 *   d_out, out_pitch H rows of out_pitch >= W elements of the image's type
 * One kernel launch, each pixel read once and written once. Returns KOHLER_OK, KOHLER_E_ARG or
 * KOHLER_E_DEVICE.
 */
int kohler_mean_image(kohler_ctx *ctx, const void *d_img, int dtype, int64_t H, int64_t W, int64_t pitch,
                      int32_t M, const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity,
                      const double *d_mean, void *d_out, int64_t out_pitch, kohler_stream_t stream);

/*
 * The k most significant thresholds (Sec. 2.1, the discussion of Fig. 1, which keeps the 6 most
 * significant local maxima; read here as the thresholds of largest contrast C): the thresholds
 * ordered by C(t) = sum(t) / count(t) descending, compared exactly (128-bit cross products), equal C
 * in ascending t; the first min(k, n) of that order. Stream-ordered, DEVICE pointers:
 *   d_sum, d_count   int64[M]: a curve (kohler_curve_async's outputs)
 *   d_thr, d_n_thr, thr_capacity   strictly ascending thresholds and their count, as for
 *                    kohler_segment; a threshold outside [0, M) counts as C = 0
 *   k                host value >= 0
 *   d_top            int32[k]: the selected thresholds, most significant first
 *   d_n_top          one int32: min(k, n)
 * One workgroup (each threshold's exact rank among the n, O(n^2) comparisons). Returns KOHLER_OK,
 * KOHLER_E_ARG or KOHLER_E_DEVICE.
 */
int kohler_top_thresholds(kohler_ctx *ctx, const int64_t *d_sum, const int64_t *d_count, int32_t M,
                          const int32_t *d_thr, const int32_t *d_n_thr, int32_t thr_capacity, int32_t k,
                          int32_t *d_top, int32_t *d_n_top, kohler_stream_t stream);

/*
 * ------------------------------------------------------------------------------------------------
 * Serving. A server runs a request loop on one context's device: callers submit images as they
 * arrive and collect each result by ticket. A scheduler thread admits queued requests in arrival
 * order whenever a device slot and enough of the image arena are free (continuous batching: work
 * that arrives while other requests are on the GPU joins the next launch, without waiting for a
 * batch to fill), and launches them on one of its streams ("lanes") as soon as a lane is idle.
 * Requests admitted together run in ONE persistent launch (the batched kernel); a request admitted
 * alone replays a HIP graph (host-to-device copy, kernel, device-to-host copy of its results) built
 * once per image shape and lane. Launches on different lanes overlap on the device. Each request's
 * difference arrays and curve stay in its slot's device memory; the server's device memory (slot
 * state plus the image arena) never exceeds hbm_budget_bytes. A request's result does not depend
 * on what it was batched with (every image is independent, Sec. 2.1).
 *
 * The family (dtype, M, nbhd) is fixed per server; launch plans come from the context (so a tuned
 * plan applies). The context must outlive the server; the server does not use the context's
 * scratch or stream, so the context stays usable for other calls.
 */
typedef struct kohler_server kohler_server;

typedef struct kohler_server_config {
    int32_t dtype, M, nbhd;    /* the family served */
    int32_t slots;             /* requests resident on the device at once (1..1024) */
    int32_t lanes;             /* streams launches go to; one launch in flight per lane (1..8) */
    int32_t max_batch;         /* most requests in one launch (1..slots) */
    int32_t queue_capacity;    /* waiting requests beyond which submit refuses (>= 1) */
    int32_t thr_capacity;      /* thresholds kept per request (0..M) */
    int32_t use_graphs;        /* nonzero: a request admitted alone replays a per-shape HIP graph
                                  (not used for requests with labels) */
    int32_t label_t0;          /* nonzero: video mode, requests may carry a label destination
                                  (kohler_server_submit_labels) */
    int64_t hbm_budget_bytes;  /* device bytes for slot state plus the image arena (> slot state) */
} kohler_server_config;

/* What happened to one request; times are CLOCK_MONOTONIC nanoseconds. */
typedef struct kohler_request_info {
    int32_t status;       /* the request's status (as kohler_curve returns it) */
    int32_t n_thresholds; /* number of local maxima (may exceed the capacity) */
    int32_t t0;
    int32_t batch;        /* requests in the launch that computed it */
    int32_t graph;        /* 1 if it ran as a graph replay */
    int32_t pad;
    int64_t t_submit_ns;  /* submit accepted the request */
    int64_t t_launch_ns;  /* admitted: the scheduler started issuing its launch */
    int64_t t_issued_ns;  /* every operation of its launch was enqueued on the lane */
    int64_t t_done_ns;    /* results in host memory, seen by the server */
} kohler_request_info;

typedef struct kohler_server_counters {
    int64_t submitted, completed, refused, cancelled;
    int64_t launches, graph_launches, batched_launches, graphs_built;
    int64_t max_batch_seen, peak_inflight;  /* peak_inflight: most requests on the device at once */
    int64_t arena_bytes, arena_peak_bytes, slot_state_bytes;
} kohler_server_counters;

/*
 * Create a server on ctx's device. Allocates, once, the slot state (per slot: accumulator replicas,
 * counters, a result record, and its pinned host mirror), the image arena (the rest of the budget)
 * and the lanes, and starts the scheduler thread. Returns KOHLER_OK, KOHLER_E_ARG (bad config or a
 * budget that does not cover the slot state), KOHLER_E_NOMEM or KOHLER_E_DEVICE.
 */
int kohler_server_create(kohler_ctx *ctx, const kohler_server_config *cfg, kohler_server **out);

/* Stop the scheduler after the launches in flight complete, drop queued requests and results not
 * yet collected, and free everything. NULL is a no-op. */
void kohler_server_destroy(kohler_server *srv);

/*
 * Submit one image (H rows of `pitch` elements of the server's dtype). A device or pinned host
 * image is read in place and must stay valid and unchanged until the request completes; a pageable
 * host image is copied into pinned staging before this returns. The server's lanes do not wait for
 * the caller's streams: a device image must be complete (every write to it finished) at submission. Returns KOHLER_OK and a ticket,
 * KOHLER_E_ARG (bad shape), or KOHLER_E_BUSY when the queue is full or the image alone exceeds the
 * image arena (then no ticket is issued).
 */
int kohler_server_submit(kohler_server *srv, const void *img, int64_t H, int64_t W, int64_t pitch,
                         uint64_t *ticket);

/*
 * Video mode (a server created with label_t0 != 0): as kohler_server_submit, and the launch that
 * computes the image's curve also segments the image in two classes at its own optimal threshold
 * t0 (eq (4); the two-class segmentation of the paper's video experiment, Sec. 4): labels[y *
 * label_pitch + x] = 1 where f(y, x) > t0, else 0, and 0 everywhere when t0 = -1 (the curve is
 * identically zero: one class). t0 never leaves the device on the way: curve, t0 and labels are one
 * stream-ordered sequence. `labels` (H rows of label_pitch >= W bytes) is device memory (written
 * there directly) or host memory (written through a block of the image arena and a copy; pinned
 * memory keeps the copy asynchronous); it must stay valid until the request completes and holds the
 * labels once kohler_server_wait returns. Returns as kohler_server_submit, and KOHLER_E_ARG when the
 * server is not in video mode.
 */
int kohler_server_submit_labels(kohler_server *srv, const void *img, int64_t H, int64_t W, int64_t pitch,
                                uint8_t *labels, int64_t label_pitch, uint64_t *ticket);

/* 1 if the request has completed (or was cancelled), 0 if not yet, KOHLER_E_ARG for an unknown
 * ticket. Never blocks. */
int kohler_server_poll(kohler_server *srv, uint64_t ticket);

/*
 * Block until the request completes, copy its results to HOST arrays (sum, count: M int64; C: M
 * doubles; thresholds: up to thr_capacity int32 — each may be NULL to skip it), fill *info (may be
 * NULL) and release the ticket (one waiter per ticket). Returns the request's status (KOHLER_OK, KOHLER_E_RANGE,
 * KOHLER_E_CAPACITY, KOHLER_E_CANCELED, KOHLER_E_DEVICE) or KOHLER_E_ARG for an unknown ticket.
 */
int kohler_server_wait(kohler_server *srv, uint64_t ticket, int64_t *sum, int64_t *count, double *C,
                       int32_t *thresholds, int32_t thr_capacity, kohler_request_info *info);

/* Cancel a request that is still queued: KOHLER_OK (its wait then returns KOHLER_E_CANCELED),
 * KOHLER_E_BUSY if it is already on the device or done, KOHLER_E_ARG for an unknown ticket. */
int kohler_server_cancel(kohler_server *srv, uint64_t ticket);

/* Hold (paused != 0) or release admission. Queued requests wait while admission is held; the
 * launches in flight complete. Returns KOHLER_OK or KOHLER_E_ARG. */
int kohler_server_pause(kohler_server *srv, int32_t paused);

/* Counters since creation. Returns KOHLER_OK or KOHLER_E_ARG. */
int kohler_server_stats(kohler_server *srv, kohler_server_counters *out);

#ifdef __cplusplus
}
#endif

#endif /* KOHLER_H */
