/*
 * Plain FP64 CPU oracle for balanced k-means geometric partitioning
 * (von Looz, Tzovas, Meyerhenke, "Balanced k-means for Parallel Geometric
 * Partitioning", arXiv:1805.01208).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Everything is IEEE binary64, round-to-nearest-even, built with
 * -ffp-contract=off and without fast-math, so every expression below is
 * evaluated exactly in the order it is written.
 *
 * What is computed, and where the paper defines it:
 *   - effective distance dist(p, c) / influence(c), Euclidean distance, not
 *     squared (Sec. 4.2 "Balancing");
 *   - assignment = exact argmin of the effective distance over ALL k centers.
 *     The Hamerly bounds (Sec. 4.3) and the bounding-box break (Sec. 4.4,
 *     Alg. 1) are exact accelerations of this argmin, so the oracle keeps no
 *     bounds and uses no boxes;
 *   - block weights, balance test, influence update with the 5% clamp
 *     (Sec. 4.2, Eq. 1, Alg. 1);
 *   - new centers as weighted means, movement delta, convergence test
 *     (Alg. 2; Sec. 4.5);
 *   - influence erosion (Sec. 4.2, the two erosion equations);
 *   - Hilbert-curve bootstrap: index, stable sort, centers at
 *     sorted[i*n/k + n/(2k)], influence 1 (Alg. 2, Sec. 4.1).
 *
 * Readings taken where the paper is silent or inconsistent:
 *   R1  Eq. (1) is applied as influence <- influence * (target/current)^(1/d),
 *       i.e. oversized blocks lose influence, as the prose of Sec. 4.2 and its
 *       derivation require (the printed fraction has the ratio inverted).
 *   R2  The per-step factor is clamped to [0.95, 1.05]; an empty block gets
 *       1.05.
 *   R3  Block weights are reset before every sweep.
 *   R4  Balanced <=> max_c weight(c) <= L_max, with
 *       L_max = (1+eps)*ceil(n/k) for unit weights (Sec. 2) and
 *       (1+eps)*W/k for node weights; target size T = W/k.
 *   R5  max_iter counts AssignAndBalance calls, max_balance_iter counts
 *       sweeps per call; after the last sweep of a call the influence has
 *       already been adapted (Alg. 1 adapts before looping).
 *   R6  deltaThreshold is absolute and the test is strict (<).
 *   R7  beta ("average cluster diameter") = mean over non-empty blocks of the
 *       diagonal of the block's axis-aligned bounding box.
 *   R8  Erosion is applied after every movement that did not converge, before
 *       the next AssignAndBalance.  alpha = 0 when delta = 0.  A switch turns
 *       it off (the influence is then kept from round to round).
 *   R9  New centers are weighted means; an empty block keeps its center.
 *   R10 Ties in the argmin go to the lowest center index.
 *   R11 Hilbert index: Skilling's transpose algorithm (J. Skilling,
 *       "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004), bits
 *       interleaved most significant level first, dimension 0 first.  Cells:
 *       q_j = min(2^m - 1, floor((x_j - lo_j) * (2^m / ext))) with ext the
 *       largest bounding-box extent (isotropic scaling); ext = 0 gives key 0.
 *   R12 Initial center i is the sorted point floor(i*n/k) + floor(n/(2k)).
 *
 * Non-uniform target block sizes (the footnote to the objective at the start
 * of Sec. 4: other block sizes than the average, e.g. for heterogeneous
 * machines):
 *   N1  The caller gives k relative sizes t_c > 0.  tsum = t_0 + t_1 + ...
 *       summed in index order; block c has target T_c = (W * t_c) / tsum.
 *   N2  L_max,c = (1+eps) * ceil((n * t_c) / tsum) for unit weights and
 *       (1+eps) * T_c for node weights; balanced <=> weight(c) <= L_max,c
 *       for every c; the influence factor is (T_c / weight(c))^(1/d) with
 *       the clamp of R2.
 *   N3  Initial center c is the sorted point
 *       floor((n * S_c) / tsum) + floor((n * t_c) / (2 tsum)), at most n-1,
 *       with S_c = t_0 + ... + t_{c-1} summed in index order: the middle of
 *       the c-th stretch of the curve when the curve is cut in proportion
 *       to the targets.
 *   N4  Imbalance is max_c weight(c) / T_c - 1.
 *   With all t_c equal and their sums exact in FP64 (small integers, dyadic
 *   fractions) these are R4, R12 and the uniform imbalance exactly (for
 *   n*k < 2^53).
 *
 * Parity pins: see tests/test_oracle_*.py.  The full multi-round trajectory
 * on large inputs has no independent pin (the paper prints no trace): parity
 * unpinned there beyond the per-step pins and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)

double oracle_lmax(int64_t n, int k, double eps, double total_weight, int unit);

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) summation: the running sum plus a correction term. */
typedef struct { double s, c; } ksum;

static void ksum_add(ksum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double ksum_get(const ksum* a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Global bounding box, per dimension. */
int oracle_bbox(int64_t n, int d, const double* const* X, double* lo, double* hi)
{
    if (n < 1 || d < 2 || d > 3) return ORC_EINVAL;
    for (int j = 0; j < d; ++j) {
        double a = X[j][0], b = X[j][0];
        for (int64_t i = 1; i < n; ++i) {
            double v = X[j][i];
            if (v < a) a = v;
            if (v > b) b = v;
        }
        lo[j] = a;
        hi[j] = b;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Hilbert index of integer cell coordinates q[0..d-1], each in [0, 2^m).
 *
 * Skilling (2004): first turn the axes into the "transposed" Hilbert index,
 * walking the levels from the coarsest: at each level, a set bit in axis i
 * inverts the lower bits of axis 0, a clear bit exchanges the lower bits of
 * axis 0 and axis i.  Then Gray-encode across the axes and undo the excess
 * rotation.  The index is the transposed form read level by level, axis 0
 * first within a level. */
uint64_t oracle_hilbert_index(const uint32_t* q, int d, int m)
{
    uint32_t x[3];
    for (int i = 0; i < d; ++i) x[i] = q[i];
    if (m <= 0) return 0;

    uint32_t top = (uint32_t)1 << (m - 1);
    for (uint32_t bit = top; bit > 1; bit >>= 1) {
        uint32_t low = bit - 1;
        for (int i = 0; i < d; ++i) {
            if (x[i] & bit) {
                x[0] ^= low;
            } else {
                uint32_t t = (x[0] ^ x[i]) & low;
                x[0] ^= t;
                x[i] ^= t;
            }
        }
    }
    for (int i = 1; i < d; ++i) x[i] ^= x[i - 1];
    uint32_t flip = 0;
    for (uint32_t bit = top; bit > 1; bit >>= 1)
        if (x[d - 1] & bit) flip ^= bit - 1;
    for (int i = 0; i < d; ++i) x[i] ^= flip;

    uint64_t key = 0;
    for (int level = m - 1; level >= 0; --level)
        for (int i = 0; i < d; ++i)
            key = (key << 1) | ((x[i] >> level) & 1u);
    return key;
}

/* Cell coordinates and Hilbert key of every point (reading R11). */
int oracle_sfc_keys(int64_t n, int d, const double* const* X, int m, uint64_t* keys)
{
    if (n < 1 || d < 2 || d > 3 || m < 1 || d * m > 63) return ORC_EINVAL;
    double lo[3], hi[3];
    oracle_bbox(n, d, X, lo, hi);
    double ext = 0.0;
    for (int j = 0; j < d; ++j)
        if (hi[j] - lo[j] > ext) ext = hi[j] - lo[j];
    if (!(ext > 0.0)) {
        memset(keys, 0, (size_t)n * sizeof(uint64_t));
        return ORC_OK;
    }
    double scale = ldexp(1.0, m) / ext;
    double cellmax = ldexp(1.0, m) - 1.0;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint32_t q[3];
        for (int j = 0; j < d; ++j) {
            double c = floor((X[j][i] - lo[j]) * scale);
            if (c > cellmax) c = cellmax;
            q[j] = (uint32_t)c;
        }
        keys[i] = oracle_hilbert_index(q, d, m);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Stable sort by key: order by (key, original index). */
typedef struct { uint64_t key; int64_t idx; } keyidx;

static int keyidx_cmp(const void* a, const void* b)
{
    const keyidx* x = (const keyidx*)a;
    const keyidx* y = (const keyidx*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
    return 0;
}

int oracle_sfc_order(int64_t n, const uint64_t* keys, int64_t* perm)
{
    keyidx* t = (keyidx*)malloc((size_t)n * sizeof(keyidx));
    if (!t) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].idx = i; }
    qsort(t, (size_t)n, sizeof(keyidx), keyidx_cmp);
    for (int64_t i = 0; i < n; ++i) perm[i] = t[i].idx;
    free(t);
    return ORC_OK;
}

/* Sum of the k target sizes in index order (reading N1). */
static double target_sum(int k, const double* t)
{
    double sum = 0.0;
    for (int c = 0; c < k; ++c) sum += t[c];
    return sum;
}

/* Sorted position of initial center c: R12, or N3 with target sizes. */
static int64_t center_position(int64_t n, int k, int64_t c, const double* t, double tsum,
                               double prefix)
{
    if (!t) return (c * n) / k + n / (2 * (int64_t)k);
    int64_t pos = (int64_t)floor(((double)n * prefix) / tsum) +
                  (int64_t)floor(((double)n * t[c]) / (2.0 * tsum));
    return pos < n - 1 ? pos : n - 1;
}

/* Per-block targets T_c and limits L_max,c (readings R4 / N1, N2).  t may be
 * NULL (uniform).  Returns 0, or ORC_EINVAL for a non-positive or
 * non-finite target size or a sum that overflows. */
int oracle_targets(int64_t n, int k, double eps, double total_weight, int unit,
                   const double* t, double* T, double* L)
{
    if (!t) {
        for (int c = 0; c < k; ++c) {
            T[c] = total_weight / (double)k;
            L[c] = oracle_lmax(n, k, eps, total_weight, unit);
        }
        return ORC_OK;
    }
    for (int c = 0; c < k; ++c)
        if (!(t[c] > 0.0) || !isfinite(t[c])) return ORC_EINVAL;
    double tsum = target_sum(k, t);
    if (!isfinite(tsum)) return ORC_EINVAL;
    for (int c = 0; c < k; ++c) {
        T[c] = (total_weight * t[c]) / tsum;
        L[c] = unit ? (1.0 + eps) * ceil(((double)n * t[c]) / tsum) : (1.0 + eps) * T[c];
    }
    return ORC_OK;
}

/* SFC bootstrap (Alg. 2): keys, stable order, centers at evenly spaced sorted
 * positions (reading R12), or at positions in proportion to target sizes
 * (reading N3; target_sizes may be NULL).  centers is [k][d] row-major.  perm
 * (sorted -> original index) and keys (original order) may be NULL. */
int oracle_init_centers_sfc(int64_t n, int d, const double* const* X, int k, int m,
                            const double* target_sizes, double* centers, int64_t* perm_out,
                            uint64_t* keys_out)
{
    if (n < 1 || d < 2 || d > 3 || k < 1 || k > n) return ORC_EINVAL;
    uint64_t* keys = keys_out ? keys_out : (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
    int64_t* perm = perm_out ? perm_out : (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!keys || !perm) return ORC_ENOMEM;
    int rc = oracle_sfc_keys(n, d, X, m, keys);
    if (rc == ORC_OK) rc = oracle_sfc_order(n, keys, perm);
    if (rc == ORC_OK) {
        double tsum = target_sizes ? target_sum(k, target_sizes) : 0.0;
        double prefix = 0.0;
        for (int64_t i = 0; i < k; ++i) {
            int64_t pos = center_position(n, k, i, target_sizes, tsum, prefix);
            for (int j = 0; j < d; ++j) centers[i * d + j] = X[j][perm[pos]];
            if (target_sizes) prefix += target_sizes[i];
        }
    }
    if (!keys_out) free(keys);
    if (!perm_out) free(perm);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Effective distance dist(p, c) / influence(c) (Sec. 4.2), evaluated in the
 * written order: ((dx*dx + dy*dy) + dz*dz), square root, divide. */
static double eff_dist(int d, const double* const* X, int64_t i, const double* c, double infl)
{
    double dx = X[0][i] - c[0];
    double dy = X[1][i] - c[1];
    double s = dx * dx + dy * dy;
    if (d == 3) {
        double dz = X[2][i] - c[2];
        s = s + dz * dz;
    }
    return sqrt(s) / infl;
}

/* Assignment (Alg. 1 inner loop without its accelerations): exact argmin over
 * all centers, lowest index on ties (R10).  best/second receive the smallest
 * and second-smallest effective distances (second = +inf when k = 1); both
 * may be NULL. */
int oracle_assign(int64_t n, int d, const double* const* X, int k, const double* centers,
                  const double* influence, int32_t* A, double* best, double* second)
{
    if (n < 1 || d < 2 || d > 3 || k < 1) return ORC_EINVAL;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double b = INFINITY, s = INFINITY;
        int32_t arg = 0;
        for (int c = 0; c < k; ++c) {
            double e = eff_dist(d, X, i, centers + (int64_t)c * d, influence[c]);
            if (e < b) {
                s = b;
                b = e;
                arg = c;
            } else if (e < s) {
                s = e;
            }
        }
        A[i] = arg;
        if (best) best[i] = b;
        if (second) second[i] = s;
    }
    return ORC_OK;
}

/* Block weights: sum of W over each block, reset on every call (R3).  Unit
 * weights (W == NULL) give exact integer counts. */
int oracle_block_weights(int64_t n, const int32_t* A, const double* W, int k, double* out)
{
    if (n < 1 || k < 1) return ORC_EINVAL;
    if (!W) {
        int64_t* cnt = (int64_t*)calloc((size_t)k, sizeof(int64_t));
        if (!cnt) return ORC_ENOMEM;
        for (int64_t i = 0; i < n; ++i) cnt[A[i]] += 1;
        for (int c = 0; c < k; ++c) out[c] = (double)cnt[c];
        free(cnt);
        return ORC_OK;
    }
    ksum* acc = (ksum*)calloc((size_t)k, sizeof(ksum));
    if (!acc) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) ksum_add(&acc[A[i]], W[i]);
    for (int c = 0; c < k; ++c) out[c] = ksum_get(&acc[c]);
    free(acc);
    return ORC_OK;
}

/* Total weight W (compensated for node weights, n for unit weights). */
double oracle_total_weight(int64_t n, const double* W)
{
    if (!W) return (double)n;
    ksum a = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) ksum_add(&a, W[i]);
    return ksum_get(&a);
}

/* L_max of the balance constraint (Sec. 2; reading R4). */
double oracle_lmax(int64_t n, int k, double eps, double total_weight, int unit)
{
    if (unit) {
        int64_t ceil_nk = (n + k - 1) / k;
        return (1.0 + eps) * (double)ceil_nk;
    }
    return (1.0 + eps) * (total_weight / (double)k);
}

/* Balance test and influence adaptation of one sweep (Alg. 1 after the
 * block sizes are known; Eq. 1 with readings R1, R2, R4).  Returns 1 when
 * balanced (influence untouched), 0 after adapting the influence. */
int oracle_balance_step(int k, int d, const double* sizes, double lmax, double target,
                        double* influence)
{
    double mx = sizes[0];
    for (int c = 1; c < k; ++c)
        if (sizes[c] > mx) mx = sizes[c];
    if (mx <= lmax) return 1;
    for (int c = 0; c < k; ++c) {
        double f;
        if (sizes[c] > 0.0) {
            double g = target / sizes[c];
            f = (d == 2) ? sqrt(g) : cbrt(g);
            if (f > 1.05) f = 1.05;
            if (f < 0.95) f = 0.95;
        } else {
            f = 1.05;
        }
        influence[c] = influence[c] * f;
    }
    return 0;
}

/* The same step with a target and a limit per block (readings N1, N2). */
int oracle_balance_step_targets(int k, int d, const double* sizes, const double* L,
                                const double* T, double* influence)
{
    int over = 0;
    for (int c = 0; c < k; ++c)
        if (sizes[c] > L[c]) over = 1;
    if (!over) return 1;
    for (int c = 0; c < k; ++c) {
        double f;
        if (sizes[c] > 0.0) {
            double g = T[c] / sizes[c];
            f = (d == 2) ? sqrt(g) : cbrt(g);
            if (f > 1.05) f = 1.05;
            if (f < 0.95) f = 0.95;
        } else {
            f = 1.05;
        }
        influence[c] = influence[c] * f;
    }
    return 0;
}

/* New centers (Alg. 2 center update; weighted mean, R9) and the distance
 * delta[c] each center moved.  centers_old/new are [k][d]. */
int oracle_new_centers(int64_t n, int d, const double* const* X, const double* W,
                       const int32_t* A, int k, const double* centers_old,
                       double* centers_new, double* delta)
{
    ksum* sx = (ksum*)calloc((size_t)k * d, sizeof(ksum));
    ksum* sw = (ksum*)calloc((size_t)k, sizeof(ksum));
    if (!sx || !sw) { free(sx); free(sw); return ORC_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) {
        int c = A[i];
        double w = W ? W[i] : 1.0;
        for (int j = 0; j < d; ++j) ksum_add(&sx[(int64_t)c * d + j], w * X[j][i]);
        ksum_add(&sw[c], w);
    }
    for (int c = 0; c < k; ++c) {
        double wsum = ksum_get(&sw[c]);
        for (int j = 0; j < d; ++j) {
            double v = centers_old[(int64_t)c * d + j];
            if (wsum > 0.0) v = ksum_get(&sx[(int64_t)c * d + j]) / wsum;
            centers_new[(int64_t)c * d + j] = v;
        }
        double dx = centers_new[(int64_t)c * d + 0] - centers_old[(int64_t)c * d + 0];
        double dy = centers_new[(int64_t)c * d + 1] - centers_old[(int64_t)c * d + 1];
        double s = dx * dx + dy * dy;
        if (d == 3) {
            double dz = centers_new[(int64_t)c * d + 2] - centers_old[(int64_t)c * d + 2];
            s = s + dz * dz;
        }
        delta[c] = sqrt(s);
    }
    free(sx);
    free(sw);
    return ORC_OK;
}

/* beta: mean bounding-box diagonal over non-empty blocks (R7). */
double oracle_beta(int64_t n, int d, const double* const* X, const int32_t* A, int k)
{
    double* lo = (double*)malloc((size_t)k * d * sizeof(double));
    double* hi = (double*)malloc((size_t)k * d * sizeof(double));
    char* seen = (char*)calloc((size_t)k, 1);
    if (!lo || !hi || !seen) { free(lo); free(hi); free(seen); return NAN; }
    for (int64_t i = 0; i < n; ++i) {
        int c = A[i];
        for (int j = 0; j < d; ++j) {
            double v = X[j][i];
            int64_t o = (int64_t)c * d + j;
            if (!seen[c] || v < lo[o]) lo[o] = v;
            if (!seen[c] || v > hi[o]) hi[o] = v;
        }
        seen[c] = 1;
    }
    ksum acc = {0.0, 0.0};
    int64_t nonempty = 0;
    for (int c = 0; c < k; ++c) {
        if (!seen[c]) continue;
        double ex = hi[(int64_t)c * d + 0] - lo[(int64_t)c * d + 0];
        double ey = hi[(int64_t)c * d + 1] - lo[(int64_t)c * d + 1];
        double s = ex * ex + ey * ey;
        if (d == 3) {
            double ez = hi[(int64_t)c * d + 2] - lo[(int64_t)c * d + 2];
            s = s + ez * ez;
        }
        ksum_add(&acc, sqrt(s));
        nonempty += 1;
    }
    free(lo);
    free(hi);
    free(seen);
    return ksum_get(&acc) / (double)nonempty;
}

/* Influence erosion (Sec. 4.2): alpha = 2/(1+exp(min(-delta/beta,0))) - 1,
 * influence <- exp((1-alpha) * log(influence)); alpha = 0 when delta = 0. */
void oracle_erode(int k, const double* delta, double beta, double* influence)
{
    for (int c = 0; c < k; ++c) {
        if (delta[c] == 0.0) continue;
        double t = -delta[c] / beta;
        if (t > 0.0) t = 0.0;
        double alpha = 2.0 / (1.0 + exp(t)) - 1.0;
        influence[c] = exp((1.0 - alpha) * log(influence[c]));
    }
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t rounds;           /* AssignAndBalance calls made */
    int32_t sweeps;           /* assignment sweeps made, all calls */
    int32_t balanced;         /* the last call ended balanced */
    int32_t converged;        /* max delta fell below the threshold */
    double imbalance;         /* max_c weight / T_c - 1 of the returned A */
    double max_block_weight;
    double lmax;              /* L_max (the largest L_max,c with target sizes) */
} oracle_info;

/* Balanced k-means (Alg. 2 around Alg. 1) with readings R1-R12.
 * centers_init ([k][d]) and influence_init ([k]) may be NULL: SFC-bootstrap
 * centers, influence 1.  k may exceed n only when the centers are given (a
 * sample round of the random-sample initialization).  target_sizes ([k]
 * relative sizes, readings N1-N4) may be NULL for equal blocks.
 * sweeps_per_round, if not NULL, receives the sweep count of every round
 * (max_iter entries). */
int oracle_balanced_kmeans(int64_t n, int d, const double* const* X, const double* W,
                           int k, double eps, int max_iter, int max_balance_iter,
                           double delta_threshold, int hilbert_order, int erosion,
                           const double* centers_init, const double* influence_init,
                           const double* target_sizes, int32_t* A,
                           double* centers_out, double* influence_out, double* block_weights_out,
                           int32_t* sweeps_per_round, oracle_info* info)
{
    if (n < 1 || d < 2 || d > 3 || k < 1 || (k > n && !centers_init) || !(eps >= 0.0) ||
        max_iter < 1 || max_balance_iter < 1)
        return ORC_EINVAL;
    int rc = ORC_OK;
    double* C = (double*)malloc((size_t)k * d * sizeof(double));
    double* Cn = (double*)malloc((size_t)k * d * sizeof(double));
    double* I = (double*)malloc((size_t)k * sizeof(double));
    double* sz = (double*)malloc((size_t)k * sizeof(double));
    double* delta = (double*)malloc((size_t)k * sizeof(double));
    double* T = (double*)malloc((size_t)k * sizeof(double));
    double* L = (double*)malloc((size_t)k * sizeof(double));
    if (!C || !Cn || !I || !sz || !delta || !T || !L) { rc = ORC_ENOMEM; goto done; }

    double wtot = oracle_total_weight(n, W);
    if ((rc = oracle_targets(n, k, eps, wtot, W == NULL, target_sizes, T, L)) != ORC_OK)
        goto done;
    if (centers_init)
        memcpy(C, centers_init, (size_t)k * d * sizeof(double));
    else if ((rc = oracle_init_centers_sfc(n, d, X, k, hilbert_order, target_sizes, C, NULL,
                                           NULL)) != ORC_OK)
        goto done;
    for (int c = 0; c < k; ++c) I[c] = influence_init ? influence_init[c] : 1.0;

    double lmax = oracle_lmax(n, k, eps, wtot, W == NULL);
    double target = wtot / (double)k;

    oracle_info inf;
    memset(&inf, 0, sizeof(inf));
    inf.lmax = L[0];
    for (int c = 1; c < k; ++c)
        if (L[c] > inf.lmax) inf.lmax = L[c];
    for (int it = 0; it < max_iter; ++it) {
        int balanced = 0, sw = 0;
        for (int b = 0; b < max_balance_iter; ++b) {
            oracle_assign(n, d, X, k, C, I, A, NULL, NULL);
            oracle_block_weights(n, A, W, k, sz);
            sw += 1;
            int bal = target_sizes ? oracle_balance_step_targets(k, d, sz, L, T, I)
                                   : oracle_balance_step(k, d, sz, lmax, target, I);
            if (bal) { balanced = 1; break; }
        }
        if (sweeps_per_round) sweeps_per_round[it] = sw;
        inf.rounds += 1;
        inf.sweeps += sw;
        inf.balanced = balanced;

        if ((rc = oracle_new_centers(n, d, X, W, A, k, C, Cn, delta)) != ORC_OK) goto done;
        double dmax = 0.0;
        for (int c = 0; c < k; ++c)
            if (delta[c] > dmax) dmax = delta[c];
        if (dmax < delta_threshold) {
            inf.converged = 1;
            memcpy(C, Cn, (size_t)k * d * sizeof(double));
            break;
        }
        if (erosion) {
            double beta = oracle_beta(n, d, X, A, k);
            oracle_erode(k, delta, beta, I);
        }
        memcpy(C, Cn, (size_t)k * d * sizeof(double));
    }

    oracle_block_weights(n, A, W, k, sz);
    inf.max_block_weight = sz[0];
    for (int c = 1; c < k; ++c)
        if (sz[c] > inf.max_block_weight) inf.max_block_weight = sz[c];
    if (target_sizes) {
        double r = sz[0] / T[0];
        for (int c = 1; c < k; ++c)
            if (sz[c] / T[c] > r) r = sz[c] / T[c];
        inf.imbalance = r - 1.0;
    } else {
        inf.imbalance = inf.max_block_weight / target - 1.0;
    }
    if (centers_out) memcpy(centers_out, C, (size_t)k * d * sizeof(double));
    if (influence_out) memcpy(influence_out, I, (size_t)k * sizeof(double));
    if (block_weights_out) memcpy(block_weights_out, sz, (size_t)k * sizeof(double));
    if (info) *info = inf;
done:
    free(C); free(Cn); free(I); free(sz); free(delta); free(T); free(L);
    return rc;
}

/* Random-sample initialization (described with Alg. 2 in Sec. 4: random
 * initialization).  The points are put in a random order, given as one key
 * per point (order by (key, index)).  Starting from the SFC centers and
 * influence 1, rounds run on the first s points of that order, s =
 * sample_start (0: 100 points per block, i.e. 100 * k, the paper's 100
 * points per process with one block per process) and doubling after
 * every round, each carrying centers and
 * influence on; once s >= n, the run on all points continues from them.
 * Each sample round is one AssignAndBalance with the sample's own balance
 * target and L_max, then one center movement with erosion (a round whose
 * movement is below delta_threshold returns its centers without erosion).
 * The sample rounds do not count towards max_iter. */
int oracle_balanced_kmeans_sampled(int64_t n, int d, const double* const* X, const double* W,
                                   int k, double eps, int max_iter, int max_balance_iter,
                                   double delta_threshold, int hilbert_order, int erosion,
                                   int64_t sample_start, const uint64_t* sample_keys,
                                   const double* target_sizes, int32_t* A, double* centers_out, double* influence_out,
                                   double* block_weights_out, int32_t* sweeps_per_round,
                                   oracle_info* info, int32_t* sample_rounds,
                                   int32_t* sample_sweeps)
{
    if (n < 1 || d < 2 || d > 3 || k < 1 || k > n || sample_start < 0 || !sample_keys)
        return ORC_EINVAL;
    if (sample_start == 0) sample_start = 100 * (int64_t)k;
    int rc = ORC_OK;
    double* C = (double*)malloc((size_t)k * d * sizeof(double));
    double* I = (double*)malloc((size_t)k * sizeof(double));
    int64_t* order = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    double* xs = (double*)malloc((size_t)n * d * sizeof(double));
    double* ws = W ? (double*)malloc((size_t)n * sizeof(double)) : NULL;
    int32_t* As = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!C || !I || !order || !xs || (W && !ws) || !As) { rc = ORC_ENOMEM; goto done; }
    if ((rc = oracle_init_centers_sfc(n, d, X, k, hilbert_order, target_sizes, C, NULL,
                                      NULL)) != ORC_OK)
        goto done;
    for (int c = 0; c < k; ++c) I[c] = 1.0;
    if ((rc = oracle_sfc_order(n, sample_keys, order)) != ORC_OK) goto done;
    int32_t rounds = 0, sweeps = 0;
    for (int64_t s = sample_start; s < n; s *= 2) {
        const double* Xs[3];
        for (int j = 0; j < d; ++j) {
            double* col = xs + (int64_t)j * n;
            for (int64_t i = 0; i < s; ++i) col[i] = X[j][order[i]];
            Xs[j] = col;
        }
        if (W)
            for (int64_t i = 0; i < s; ++i) ws[i] = W[order[i]];
        oracle_info si;
        rc = oracle_balanced_kmeans(s, d, Xs, ws, k, eps, 1, max_balance_iter, delta_threshold,
                                    hilbert_order, erosion, C, I, target_sizes, As, C, I, NULL,
                                    NULL, &si);
        if (rc != ORC_OK) goto done;
        rounds += 1;
        sweeps += si.sweeps;
    }
    if (sample_rounds) *sample_rounds = rounds;
    if (sample_sweeps) *sample_sweeps = sweeps;
    rc = oracle_balanced_kmeans(n, d, X, W, k, eps, max_iter, max_balance_iter, delta_threshold,
                                hilbert_order, erosion, C, I, target_sizes, A, centers_out,
                                influence_out,
                                block_weights_out, sweeps_per_round, info);
done:
    free(C); free(I); free(order); free(xs); free(ws); free(As);
    return rc;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    double imbalance;        /* max_c weight / T_c - 1 */
    double objective;        /* sum_p w(p) * dist(p, mean of its block)^2 */
    double lmax;             /* L_max (the largest L_max,c with target sizes) */
    int32_t empty_blocks;
    int32_t overloaded_blocks;  /* weight > L_max,c (Sec. 2 "overloaded") */
} oracle_stats;

/* Partition statistics of a given assignment: block weights, block means
 * (NaN for an empty block), imbalance, k-means objective; target_sizes may
 * be NULL (equal blocks; readings N1, N2, N4 otherwise). */
int oracle_partition_stats(int64_t n, int d, const double* const* X, const double* W,
                           const int32_t* A, int k, double eps, const double* target_sizes,
                           double* block_weights, double* centers, oracle_stats* st)
{
    if (n < 1 || d < 2 || d > 3 || k < 1) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (A[i] < 0 || A[i] >= k) return ORC_EINVAL;
    double* bw = (double*)malloc((size_t)k * sizeof(double));
    double* C = (double*)malloc((size_t)k * d * sizeof(double));
    double* C0 = (double*)calloc((size_t)k * d, sizeof(double));
    double* dl = (double*)malloc((size_t)k * sizeof(double));
    double* T = (double*)malloc((size_t)k * sizeof(double));
    double* L = (double*)malloc((size_t)k * sizeof(double));
    if (!bw || !C || !C0 || !dl || !T || !L) {
        free(bw); free(C); free(C0); free(dl); free(T); free(L);
        return ORC_ENOMEM;
    }
    double wtot = oracle_total_weight(n, W);
    if (oracle_targets(n, k, eps, wtot, W == NULL, target_sizes, T, L) != ORC_OK) {
        free(bw); free(C); free(C0); free(dl); free(T); free(L);
        return ORC_EINVAL;
    }
    oracle_block_weights(n, A, W, k, bw);
    oracle_new_centers(n, d, X, W, A, k, C0, C, dl);
    double ratio = bw[0] / T[0], lmax = L[0];
    int32_t empty = 0, over = 0;
    for (int c = 0; c < k; ++c) {
        if (bw[c] / T[c] > ratio) ratio = bw[c] / T[c];
        if (L[c] > lmax) lmax = L[c];
        if (bw[c] == 0.0) {
            empty += 1;
            for (int j = 0; j < d; ++j) C[(int64_t)c * d + j] = NAN;
        }
        if (bw[c] > L[c]) over += 1;
    }
    ksum obj = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        const double* c = C + (int64_t)A[i] * d;
        double dx = X[0][i] - c[0];
        double dy = X[1][i] - c[1];
        double s = dx * dx + dy * dy;
        if (d == 3) {
            double dz = X[2][i] - c[2];
            s = s + dz * dz;
        }
        ksum_add(&obj, (W ? W[i] : 1.0) * s);
    }
    st->imbalance = ratio - 1.0;
    st->objective = ksum_get(&obj);
    st->lmax = lmax;
    st->empty_blocks = empty;
    st->overloaded_blocks = over;
    if (block_weights) memcpy(block_weights, bw, (size_t)k * sizeof(double));
    if (centers) memcpy(centers, C, (size_t)k * d * sizeof(double));
    free(bw); free(C); free(C0); free(dl); free(T); free(L);
    return ORC_OK;
}

/* Threads the OpenMP parts use (for reporting the CPU baseline). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
