/*
 * Köhler contrast curve: CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this file; only the
 * test suite, the smoke check and the bench's CPU-baseline leg do. It shares no code with the HIP
 * implementation.
 *
 * Reference: G. Noyel, "Speeding up the Köhler's method of contrast thresholding" (arXiv 1707.05062).
 *
 * The image is a function f on a rectangular domain D (H rows, W columns, row-major, contiguous)
 * with integer values in [0, M). Thresholds t are the integers 0..M-1 (Sec. 2.1).
 *
 *   oracle_curve   the definition itself (Sec. 2.1, eqs (1)-(3)): for each threshold t, list the
 *                  boundary B(t) = ordered pairs (x0, x1) of neighbours with f(x0) <= t < f(x1),
 *                  over the FULL 4- or 8-neighbourhood, add up min(f(x1)-t, t-f(x0)) and the pair
 *                  count, and divide. O(M * N * |A|). It never uses the half-neighbourhood result
 *                  of Sec. 3.2 (eq (9)), so agreeing with it checks that theorem too.
 *   oracle_alg1    the paper's fast algorithm (Sec. 3.1, Algorithm 1) written from its description:
 *                  visit every unordered neighbour pair once through the half neighbourhood, and
 *                  add the pair's contrast to every threshold between its two grey levels. A
 *                  structurally different exact route to the same integers.
 *   oracle_thresholds  local maxima of the curve and the optimal threshold of eq (4), with exact
 *                  rational comparisons of the curve values.
 *   oracle_curve_nbhd, oracle_alg1_nbhd  the same two routes for other neighbourhoods: Sec. 2.1
 *                  allows the 6-neighbourhood besides N4 and N8, and the argument of Sec. 3.2 (eqs
 *                  (7)-(9)) holds for any symmetric structuring element A (a in A <=> -a in A) and a
 *                  half A* holding one offset of each pair {a, -a}. Two kinds:
 *                    generic  a symmetric offset set A, the same at every pixel;
 *                    hex      the 6-neighbourhood of a hexagonal grid stored on the H x W raster with
 *                             the odd rows shifted right by half a pixel: a pixel of an even row y has
 *                             the neighbours (y, x-1), (y, x+1), (y-1, x-1), (y-1, x), (y+1, x-1),
 *                             (y+1, x); a pixel of an odd row (y, x-1), (y, x+1), (y-1, x), (y-1, x+1),
 *                             (y+1, x), (y+1, x+1). The relation is symmetric, though not the same
 *                             offsets at every pixel.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - pairs exist only when both pixels lie in D: no wrap-around, no padding pairs;
 *   - C(t) = 0 where B(t) is empty (the paper divides by #B(t) without a guard);
 *   - sum and count are exact int64; C(t) is one IEEE binary64 division of the two;
 *   - a local maximum is a maximal run [a, b] of equal positive C whose neighbours on both sides
 *     (where they exist) are strictly smaller; it is reported at a, the run's first threshold;
 *   - t0 is the smallest threshold attaining the maximum of C, or -1 when C is identically zero.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_RANGE (-2)
#define ORACLE_E_CAPACITY (-3)

/* Full neighbourhoods as (row, column) offsets: N4 first, then the four diagonals of N8. */
static const int NB_DY[8] = {-1, 1, 0, 0, -1, -1, 1, 1};
static const int NB_DX[8] = {0, 0, -1, 1, -1, 1, -1, 1};

/* Half neighbourhoods (Sec. 3.2): one offset of each symmetric pair {a, -a}. */
static const int HALF_DY[4] = {0, 1, 1, 1};
static const int HALF_DX[4] = {1, 0, 1, -1};

static int check_args(const int32_t *f, int64_t H, int64_t W, int32_t M, int32_t nbhd)
{
    if (!f || H < 1 || W < 1 || M < 1 || (nbhd != 4 && nbhd != 8))
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < H * W; i++)
        if (f[i] < 0 || f[i] >= M)
            return ORACLE_E_RANGE;
    return ORACLE_OK;
}

/*
 * Eqs (1)-(3) for the thresholds ts[0..nts-1]: sum[k] = sum of C_K^t over B(t), count[k] = #B(t),
 * C[k] = sum[k] / count[k] (0 when B(t) is empty), with t = ts[k]. Parallel over thresholds.
 */
int oracle_curve(const int32_t *f, int64_t H, int64_t W, int32_t M, int32_t nbhd,
                 const int32_t *ts, int32_t nts, int64_t *sum, int64_t *count, double *C)
{
    int st = check_args(f, H, W, M, nbhd);
    if (st != ORACLE_OK)
        return st;
    if (!ts || nts < 0 || !sum || !count || !C)
        return ORACLE_E_ARG;
    for (int32_t k = 0; k < nts; k++)
        if (ts[k] < 0 || ts[k] >= M)
            return ORACLE_E_ARG;

#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < nts; k++) {
        const int64_t t = ts[k];
        int64_t S = 0, K = 0;
        for (int64_t y = 0; y < H; y++) {
            for (int64_t x = 0; x < W; x++) {
                const int64_t f0 = f[y * W + x];
                if (f0 > t) /* x0 must lie in C_0^t */
                    continue;
                for (int a = 0; a < nbhd; a++) {
                    const int64_t y1 = y + NB_DY[a], x1 = x + NB_DX[a];
                    if (y1 < 0 || y1 >= H || x1 < 0 || x1 >= W) /* x1 must lie in D */
                        continue;
                    const int64_t f1 = f[y1 * W + x1];
                    if (f1 <= t) /* x1 must lie in C_1^t */
                        continue;
                    const int64_t up = f1 - t, down = t - f0; /* eq (2) */
                    S += up < down ? up : down;
                    K += 1;
                }
            }
        }
        sum[k] = S;
        count[k] = K;
        C[k] = K ? (double)S / (double)K : 0.0;
    }
    return ORACLE_OK;
}

/*
 * Algorithm 1 (Sec. 3.1) with the half neighbourhood of Sec. 3.2: each unordered neighbour pair
 * {p, q} is seen once; with lo = min(f_p, f_q) and hi = max(f_p, f_q) it belongs to B(t) exactly
 * for lo <= t < hi, where its contrast is min(hi - t, t - lo). Rows are split across threads, each
 * with private accumulators that are summed at the end (Sec. 3.3).
 */
int oracle_alg1(const int32_t *f, int64_t H, int64_t W, int32_t M, int32_t nbhd,
                int64_t *sum, int64_t *count)
{
    int st = check_args(f, H, W, M, nbhd);
    if (st != ORACLE_OK)
        return st;
    if (!sum || !count)
        return ORACLE_E_ARG;
    const int nhalf = nbhd / 2;
    memset(sum, 0, sizeof(int64_t) * (size_t)M);
    memset(count, 0, sizeof(int64_t) * (size_t)M);

#pragma omp parallel
    {
        int64_t *ps = (int64_t *)calloc((size_t)M, sizeof(int64_t));
        int64_t *pk = (int64_t *)calloc((size_t)M, sizeof(int64_t));
#pragma omp for schedule(static)
        for (int64_t y = 0; y < H; y++) {
            for (int a = 0; a < nhalf; a++) {
                const int64_t y1 = y + HALF_DY[a];
                if (y1 >= H)
                    continue;
                for (int64_t x = 0; x < W; x++) {
                    const int64_t x1 = x + HALF_DX[a];
                    if (x1 < 0 || x1 >= W)
                        continue;
                    const int64_t p = f[y * W + x], q = f[y1 * W + x1];
                    const int64_t lo = p < q ? p : q, hi = p < q ? q : p;
                    for (int64_t t = lo; t < hi; t++) {
                        const int64_t up = hi - t, down = t - lo;
                        ps[t] += up < down ? up : down;
                        pk[t] += 1;
                    }
                }
            }
        }
#pragma omp critical
        for (int32_t t = 0; t < M; t++) {
            sum[t] += ps[t];
            count[t] += pk[t];
        }
        free(ps);
        free(pk);
    }
    return ORACLE_OK;
}

/* sign(C(u) - C(v)) computed exactly: C = s / k, or 0 when k = 0. Products fit in 128 bits. */
static int cmp_curve(int64_t su, int64_t ku, int64_t sv, int64_t kv)
{
    const __int128 nu = ku ? su : 0, du = ku ? ku : 1;
    const __int128 nv = kv ? sv : 0, dv = kv ? kv : 1;
    const __int128 l = nu * dv, r = nv * du;
    return (l > r) - (l < r);
}

/*
 * Local maxima of C (ascending) and t0 of eq (4). thr receives at most cap entries; *n gets the
 * full number found, and ORACLE_E_CAPACITY is returned when it exceeds cap.
 */
int oracle_thresholds(const int64_t *sum, const int64_t *count, int32_t M,
                      int32_t *thr, int32_t cap, int32_t *n, int32_t *t0)
{
    if (!sum || !count || M < 1 || cap < 0 || (cap > 0 && !thr) || !n || !t0)
        return ORACLE_E_ARG;

    int32_t found = 0;
    int32_t a = 0;
    while (a < M) {
        int32_t b = a; /* extend the run of equal values [a, b] */
        while (b + 1 < M && cmp_curve(sum[b + 1], count[b + 1], sum[a], count[a]) == 0)
            b++;
        const int positive = cmp_curve(sum[a], count[a], 0, 1) > 0;
        const int left_ok = a == 0 || cmp_curve(sum[a - 1], count[a - 1], sum[a], count[a]) < 0;
        const int right_ok = b == M - 1 || cmp_curve(sum[b + 1], count[b + 1], sum[b], count[b]) < 0;
        if (positive && left_ok && right_ok) {
            if (found < cap)
                thr[found] = a;
            found++;
        }
        a = b + 1;
    }
    *n = found;

    int32_t best = 0;
    for (int32_t t = 1; t < M; t++)
        if (cmp_curve(sum[t], count[t], sum[best], count[best]) > 0)
            best = t;
    *t0 = cmp_curve(sum[best], count[best], 0, 1) > 0 ? best : -1;
    return found > cap ? ORACLE_E_CAPACITY : ORACLE_OK;
}

/* ------------------------------------------------------------------------------------------------
 * Other neighbourhoods (Sec. 2.1; Sec. 3.2 eqs (7)-(9) for a symmetric structuring element).
 */
#define ORACLE_MAX_OFFSETS 64

static int check_image(const int32_t *f, int64_t H, int64_t W, int32_t M)
{
    if (!f || H < 1 || W < 1 || M < 1)
        return ORACLE_E_ARG;
    for (int64_t i = 0; i < H * W; i++)
        if (f[i] < 0 || f[i] >= M)
            return ORACLE_E_RANGE;
    return ORACLE_OK;
}

/* The hexagonal grid's neighbour offsets of a pixel in row y (odd rows shifted right). */
static void hex_full(int64_t y, int *ody, int *odx)
{
    static const int EY[6] = {0, 0, -1, -1, 1, 1}, EX[6] = {-1, 1, -1, 0, -1, 0};
    static const int OY[6] = {0, 0, -1, -1, 1, 1}, OX[6] = {-1, 1, 0, 1, 0, 1};
    const int odd = (int)(y & 1);
    for (int a = 0; a < 6; a++) {
        ody[a] = odd ? OY[a] : EY[a];
        odx[a] = odd ? OX[a] : EX[a];
    }
}

/* A symmetric offset set: 1..64 distinct non-zero offsets, with -a present for every a. */
static int check_symmetric(const int32_t *dy, const int32_t *dx, int32_t n)
{
    if (!dy || !dx || n < 1 || n > ORACLE_MAX_OFFSETS)
        return ORACLE_E_ARG;
    for (int32_t a = 0; a < n; a++) {
        if (dy[a] == 0 && dx[a] == 0)
            return ORACLE_E_ARG;
        int mirrored = 0;
        for (int32_t b = 0; b < n; b++) {
            if (b != a && dy[b] == dy[a] && dx[b] == dx[a])
                return ORACLE_E_ARG;
            if (dy[b] == -dy[a] && dx[b] == -dx[a])
                mirrored = 1;
        }
        if (!mirrored)
            return ORACLE_E_ARG;
    }
    return ORACLE_OK;
}

/*
 * Eqs (1)-(3) over the full neighbourhood (hex != 0: the hexagonal rule, dy/dx/n unused; else the
 * symmetric set A = {(dy[a], dx[a])}): ordered pairs (x0, x1), x1 a neighbour of x0 inside D,
 * f(x0) <= t < f(x1), contrast min(f(x1) - t, t - f(x0)).
 */
int oracle_curve_nbhd(const int32_t *f, int64_t H, int64_t W, int32_t M, const int32_t *dy,
                      const int32_t *dx, int32_t n, int32_t hex, const int32_t *ts, int32_t nts,
                      int64_t *sum, int64_t *count, double *C)
{
    int st = check_image(f, H, W, M);
    if (st != ORACLE_OK)
        return st;
    if (!hex && check_symmetric(dy, dx, n) != ORACLE_OK)
        return ORACLE_E_ARG;
    if (!ts || nts < 0 || !sum || !count || !C)
        return ORACLE_E_ARG;
    for (int32_t k = 0; k < nts; k++)
        if (ts[k] < 0 || ts[k] >= M)
            return ORACLE_E_ARG;

#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < nts; k++) {
        const int64_t t = ts[k];
        int64_t S = 0, K = 0;
        int ody[ORACLE_MAX_OFFSETS], odx[ORACLE_MAX_OFFSETS];
        for (int64_t y = 0; y < H; y++) {
            int na = (int)n;
            if (hex) {
                hex_full(y, ody, odx);
                na = 6;
            } else {
                for (int a = 0; a < na; a++) {
                    ody[a] = dy[a];
                    odx[a] = dx[a];
                }
            }
            for (int64_t x = 0; x < W; x++) {
                const int64_t f0 = f[y * W + x];
                if (f0 > t) /* x0 in C_0^t */
                    continue;
                for (int a = 0; a < na; a++) {
                    const int64_t y1 = y + ody[a], x1 = x + odx[a];
                    if (y1 < 0 || y1 >= H || x1 < 0 || x1 >= W) /* x1 in D */
                        continue;
                    const int64_t f1 = f[y1 * W + x1];
                    if (f1 <= t) /* x1 in C_1^t */
                        continue;
                    const int64_t rise = f1 - t, fall = t - f0; /* eq (2) */
                    S += rise < fall ? rise : fall;
                    K++;
                }
            }
        }
        sum[k] = S;
        count[k] = K;
        C[k] = K > 0 ? (double)S / (double)K : 0.0;
    }
    return ORACLE_OK;
}

/*
 * Algorithm 1 over a half neighbourhood: every unordered pair {p, p + a}, a in the half set,
 * counted once for lo <= t < hi with contrast min(hi - t, t - lo). hex != 0: the half of the
 * hexagonal rule, (0, 1) and the two neighbours in the row below ((1, -1), (1, 0) for an even row,
 * (1, 0), (1, 1) for an odd one); else the given half set, which must hold no offset together with
 * its negation.
 */
int oracle_alg1_nbhd(const int32_t *f, int64_t H, int64_t W, int32_t M, const int32_t *hdy,
                     const int32_t *hdx, int32_t nh, int32_t hex, int64_t *sum, int64_t *count)
{
    int st = check_image(f, H, W, M);
    if (st != ORACLE_OK)
        return st;
    if (!sum || !count)
        return ORACLE_E_ARG;
    if (!hex) {
        if (!hdy || !hdx || nh < 1 || nh > ORACLE_MAX_OFFSETS)
            return ORACLE_E_ARG;
        for (int32_t a = 0; a < nh; a++) {
            if (hdy[a] == 0 && hdx[a] == 0)
                return ORACLE_E_ARG;
            for (int32_t b = 0; b < nh; b++) {
                if (b != a && hdy[b] == hdy[a] && hdx[b] == hdx[a])
                    return ORACLE_E_ARG;
                if (hdy[b] == -hdy[a] && hdx[b] == -hdx[a])
                    return ORACLE_E_ARG;
            }
        }
    }
    static const int HEY[3] = {0, 1, 1}, HEX_[3] = {1, -1, 0};
    static const int HOY[3] = {0, 1, 1}, HOX[3] = {1, 0, 1};
    memset(sum, 0, sizeof(int64_t) * (size_t)M);
    memset(count, 0, sizeof(int64_t) * (size_t)M);
    for (int64_t y = 0; y < H; y++) {
        const int na = hex ? 3 : (int)nh;
        for (int a = 0; a < na; a++) {
            const int64_t ay = hex ? ((y & 1) ? HOY[a] : HEY[a]) : hdy[a];
            const int64_t ax = hex ? ((y & 1) ? HOX[a] : HEX_[a]) : hdx[a];
            const int64_t y1 = y + ay;
            if (y1 < 0 || y1 >= H)
                continue;
            for (int64_t x = 0; x < W; x++) {
                const int64_t x1 = x + ax;
                if (x1 < 0 || x1 >= W)
                    continue;
                const int64_t p = f[y * W + x], q = f[y1 * W + x1];
                const int64_t lo = p < q ? p : q, hi = p < q ? q : p;
                for (int64_t t = lo; t < hi; ++t) { /* lo <= t < hi */
                    const int64_t up = hi - t, down = t - lo;
                    sum[t] += up < down ? up : down;
                    count[t] += 1;
                }
            }
        }
    }
    return ORACLE_OK;
}
