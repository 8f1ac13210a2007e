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
