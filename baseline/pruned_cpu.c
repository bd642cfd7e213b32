/*
 * Pruned FP64 balanced k-means on the host (C11, OpenMP): a CPU baseline the
 * GPU path is timed against.  It is neither the oracle nor part of the
 * product path: it computes the oracle's result -- the same loop (Alg. 2
 * around Alg. 1, readings R1-R10), the same FP64 effective distance
 * sqrt(((dx*dx + dy*dy) + dz*dz)) / influence with ties to the lower index --
 * with the paper's two exact accelerations:
 *   * per-point Hamerly bounds (Sec. 4.3): an upper bound on the effective
 *     distance to the own center and a lower bound on the second-best one;
 *     a point whose upper bound is below its lower bound keeps its block.
 *     Bounds are relaxed, not tightened, when centers move or influences
 *     change (Eqs. 2-3 read as relaxations): the upper bound is stored as a
 *     distance minus the accumulated movement of the point's center, the
 *     lower bound in a global affine frame lb = M * stored - E;
 *   * bounding-box candidates (Sec. 4.4): points are ordered along a Morton
 *     curve and cut into tiles of 1024; a center whose smallest effective
 *     distance to a tile's box exceeds the second-smallest largest one can be
 *     neither best nor second-best of any point of the tile and is not
 *     evaluated there (a 16-tile super-tile level filters the k centers
 *     first).
 * Unit weights only.  Every quantity that decides an assignment is the
 * oracle's, so the assignments, sweep counts and influences equal the
 * oracle's; centers use the same compensated sums in input order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PC_OK 0
#define PC_EINVAL (-1)
#define PC_ENOMEM (-3)
#define TILE 1024
#define SUPER 16
#define SLACK 1e-12

typedef struct {
    int32_t rounds, sweeps, balanced, converged;
    int64_t evaluated, skipped, cand_evals;
    double sweep_seconds;     /* wall time of the sweeps (candidates, assignment, counts, balance) */
    double total_seconds;     /* wall time of the whole call */
} pruned_info;

typedef struct { double s, c; } nsum;

static void nsum_add(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

typedef struct { uint64_t key; int64_t idx; } kidx;

static int kidx_cmp(const void* a, const void* b)
{
    const kidx* x = (const kidx*)a;
    const kidx* y = (const kidx*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Morton key of a point: 16 bits per axis over the bounding box. */
static uint64_t morton(int d, const double* q, const double* lo, double scale)
{
    uint64_t key = 0;
    uint32_t cell[3] = {0, 0, 0};
    for (int j = 0; j < d; ++j) {
        double v = (q[j] - lo[j]) * scale;
        uint32_t c = v <= 0.0 ? 0u : (v >= 65535.0 ? 65535u : (uint32_t)v);
        cell[j] = c;
    }
    for (int b = 15; b >= 0; --b)
        for (int j = 0; j < d; ++j) key = (key << 1) | ((cell[j] >> b) & 1u);
    return key;
}

/* Smallest and largest squared effective distance from center c to a box. */
static void box_eff2(int d, const double* blo, const double* bhi, const double* C, double iv,
                     double* lo2, double* hi2)
{
    double mn = 0.0, mx = 0.0;
    for (int j = 0; j < d; ++j) {
        double g = fmax(fmax(blo[j] - C[j], C[j] - bhi[j]), 0.0);
        double f = fmax(fabs(C[j] - blo[j]), fabs(C[j] - bhi[j]));
        mn += g * g;
        mx += f * f;
    }
    *lo2 = mn * iv * iv;
    *hi2 = mx * iv * iv;
}

/* Centers of `list` (all k when list is NULL) that can be best or second
 * best for a point in the box; returns the count, *thr the second-smallest
 * largest squared effective distance. */
static int box_filter(int d, const double* blo, const double* bhi, const double* C,
                      const double* iv, const int* list, int L, int* out, double* thr)
{
    double a = INFINITY, b = INFINITY;
    for (int i = 0; i < L; ++i) {
        int c = list ? list[i] : i;
        double lo2, hi2;
        box_eff2(d, blo, bhi, C + (int64_t)c * d, iv[c], &lo2, &hi2);
        if (hi2 < a) { b = a; a = hi2; } else if (hi2 < b) { b = hi2; }
    }
    double t = b * (1.0 + 2e-9);
    int m = 0;
    for (int i = 0; i < L; ++i) {
        int c = list ? list[i] : i;
        double lo2, hi2;
        box_eff2(d, blo, bhi, C + (int64_t)c * d, iv[c], &lo2, &hi2);
        if (lo2 <= t) out[m++] = c;
    }
    *thr = b;
    return m;
}

static void box_of(int d, double* const* xs, int64_t a, int64_t b, double* blo, double* bhi)
{
    for (int j = 0; j < d; ++j) {
        blo[j] = INFINITY;
        bhi[j] = -INFINITY;
        for (int64_t i = a; i < b; ++i) {
            blo[j] = fmin(blo[j], xs[j][i]);
            bhi[j] = fmax(bhi[j], xs[j][i]);
        }
    }
}

int pruned_balanced_kmeans(int64_t n, int d, const double* const* X, int k, double eps,
                           int max_iter, int max_balance_iter, double delta_threshold,
                           int erosion, const double* centers_init, int32_t* A_out,
                           double* centers_out, double* influence_out, pruned_info* info)
{
    if (n < 1 || d < 2 || d > 3 || k < 1 || k > n || !(eps >= 0.0) || max_iter < 1 ||
        max_balance_iter < 1 || !centers_init || !A_out)
        return PC_EINVAL;
    const double t_start = omp_get_wtime();
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int64_t nsuper = (ntiles + SUPER - 1) / SUPER;
    int rc = PC_OK;
    kidx* ord = (kidx*)malloc((size_t)n * sizeof(kidx));
    int64_t* perm = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    double* xs[3] = {NULL, NULL, NULL};
    for (int j = 0; j < d; ++j) xs[j] = (double*)malloc((size_t)n * sizeof(double));
    int32_t* A = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* Ain = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    double* ub = (double*)malloc((size_t)n * sizeof(double));
    double* lb = (double*)malloc((size_t)n * sizeof(double));
    double* tbox = (double*)malloc((size_t)ntiles * 2 * d * sizeof(double));
    double* sbox = (double*)malloc((size_t)nsuper * 2 * d * sizeof(double));
    int* slist = (int*)malloc((size_t)nsuper * k * sizeof(int));
    int* scnt = (int*)malloc((size_t)nsuper * sizeof(int));
    double* C = (double*)malloc((size_t)k * d * sizeof(double));
    double* Cn = (double*)malloc((size_t)k * d * sizeof(double));
    double* I = (double*)malloc((size_t)k * sizeof(double));
    double* iv = (double*)malloc((size_t)k * sizeof(double));
    double* Dm = (double*)calloc((size_t)k, sizeof(double));
    double* delta = (double*)malloc((size_t)k * sizeof(double));
    int64_t* cnt = (int64_t*)malloc((size_t)k * sizeof(int64_t));
    const int nth = omp_get_max_threads();
    int64_t* tcnt = (int64_t*)calloc((size_t)nth * k, sizeof(int64_t));
    if (!ord || !perm || !xs[0] || !xs[1] || (d == 3 && !xs[2]) || !A || !Ain || !ub || !lb ||
        !tbox || !sbox || !slist || !scnt || !C || !Cn || !I || !iv || !Dm || !delta || !cnt ||
        !tcnt) {
        rc = PC_ENOMEM;
        goto done;
    }

    /* Morton order and the tiles */
    double lo[3], ext = 0.0;
    for (int j = 0; j < d; ++j) {
        double mn = INFINITY, mx = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            mn = fmin(mn, X[j][i]);
            mx = fmax(mx, X[j][i]);
        }
        lo[j] = mn;
        ext = fmax(ext, mx - mn);
    }
    const double scale = ext > 0.0 ? 65535.0 / ext : 0.0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double q[3];
        for (int j = 0; j < d; ++j) q[j] = X[j][i];
        ord[i].key = morton(d, q, lo, scale);
        ord[i].idx = i;
    }
    qsort(ord, (size_t)n, sizeof(kidx), kidx_cmp);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = ord[i].idx;
        for (int j = 0; j < d; ++j) xs[j][i] = X[j][ord[i].idx];
    }
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t a = t * TILE, b = a + TILE < n ? a + TILE : n;
        box_of(d, xs, a, b, tbox + t * 2 * d, tbox + t * 2 * d + d);
    }
    for (int64_t s = 0; s < nsuper; ++s) {
        double* sb = sbox + s * 2 * d;
        for (int j = 0; j < d; ++j) {
            sb[j] = INFINITY;
            sb[d + j] = -INFINITY;
        }
        for (int64_t t = s * SUPER; t < (s + 1) * SUPER && t < ntiles; ++t)
            for (int j = 0; j < d; ++j) {
                sb[j] = fmin(sb[j], tbox[t * 2 * d + j]);
                sb[d + j] = fmax(sb[d + j], tbox[t * 2 * d + d + j]);
            }
    }

    memcpy(C, centers_init, (size_t)k * d * sizeof(double));
    for (int c = 0; c < k; ++c) {
        I[c] = 1.0;
        iv[c] = 1.0;
    }
    for (int64_t i = 0; i < n; ++i) {
        A[i] = -1;
        ub[i] = INFINITY;
        lb[i] = 0.0;
    }
    double M = 1.0, E = 0.0;
    const int64_t ceil_nk = (n + k - 1) / k;
    const double lmax = (1.0 + eps) * (double)ceil_nk;
    const double target = (double)n / (double)k;
    const double thr = delta_threshold < 0.0 ? 1e-5 * ext : delta_threshold;

    pruned_info inf;
    memset(&inf, 0, sizeof(inf));
    double tsweep = 0.0;
    for (int it = 0; it < max_iter; ++it) {
        int balanced = 0, sw = 0;
        for (int bi = 0; bi < max_balance_iter; ++bi) {
            const double t0 = omp_get_wtime();
            /* super-tile lists against all centers */
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t s = 0; s < nsuper; ++s) {
                double t;
                scnt[s] = box_filter(d, sbox + s * 2 * d, sbox + s * 2 * d + d, C, iv, NULL, k,
                                     slist + s * k, &t);
            }
            int64_t ev = 0, sk = 0, ce = 0;
            memset(tcnt, 0, (size_t)nth * k * sizeof(int64_t));
#pragma omp parallel reduction(+ : ev, sk, ce)
            {
                int* list = (int*)malloc((size_t)k * sizeof(int));
                int64_t* my = tcnt + (int64_t)omp_get_thread_num() * k;
#pragma omp for schedule(dynamic, 8)
                for (int64_t t = 0; t < ntiles; ++t) {
                    const int64_t s = t / SUPER;
                    double t2;
                    const int L = box_filter(d, tbox + t * 2 * d, tbox + t * 2 * d + d, C, iv,
                                             slist + s * k, scnt[s], list, &t2);
                    const double lb_out = sqrt(t2) * (1.0 - SLACK);
                    const int64_t a0 = t * TILE, a1 = a0 + TILE < n ? a0 + TILE : n;
                    for (int64_t i = a0; i < a1; ++i) {
                        int a = A[i];
                        if (a >= 0) {
                            /* Hamerly test, FP64 with relative slack */
                            double u = ((ub[i] + Dm[a]) + 4e-16 * (fabs(ub[i]) + Dm[a])) *
                                       iv[a] * (1.0 + SLACK);
                            double l = M * lb[i] * (1.0 - SLACK) - E * (1.0 + SLACK);
                            if (u < l) {
                                ++sk;
                                my[a] += 1;
                                continue;
                            }
                        }
                        ++ev;
                        ce += L;
                        double b = INFINITY, s2 = INFINITY, bd = INFINITY;
                        int32_t arg = 0x7fffffff;
                        for (int m = 0; m < L; ++m) {
                            const int c = list[m];
                            const double* cc = C + (int64_t)c * d;
                            double dx = xs[0][i] - cc[0];
                            double dy = xs[1][i] - cc[1];
                            double q = dx * dx + dy * dy;
                            if (d == 3) {
                                double dz = xs[2][i] - cc[2];
                                q = q + dz * dz;
                            }
                            double dist = sqrt(q);
                            double e = dist / I[c];
                            if (e < b || (e == b && c < arg)) {
                                s2 = b;
                                b = e;
                                arg = c;
                                bd = dist;
                            } else if (e < s2) {
                                s2 = e;
                            }
                        }
                        A[i] = arg;
                        my[arg] += 1;
                        ub[i] = bd * (1.0 + SLACK) - Dm[arg];
                        double lv = (fmin(s2, lb_out) + E) / M;
                        lb[i] = lv > 0.0 ? lv * (1.0 - SLACK) : 0.0;
                    }
                }
                free(list);
            }
            for (int c = 0; c < k; ++c) {
                int64_t v = 0;
                for (int q = 0; q < nth; ++q) v += tcnt[(int64_t)q * k + c];
                cnt[c] = v;
            }
            inf.evaluated += ev;
            inf.skipped += sk;
            inf.cand_evals += ce;
            sw += 1;
            /* balance test and influence update (Eq. 1 as R1, clamp R2) */
            int64_t mx = cnt[0];
            for (int c = 1; c < k; ++c)
                if (cnt[c] > mx) mx = cnt[c];
            if ((double)mx <= lmax) {
                balanced = 1;
                tsweep += omp_get_wtime() - t0;
                break;
            }
            double mu = INFINITY;
            for (int c = 0; c < k; ++c) {
                double f;
                double s = (double)cnt[c];
                if (s > 0.0) {
                    double g = target / s;
                    f = (d == 2) ? sqrt(g) : cbrt(g);
                    if (f > 1.05) f = 1.05;
                    if (f < 0.95) f = 0.95;
                } else {
                    f = 1.05;
                }
                double in = I[c] * f;
                mu = fmin(mu, I[c] / in);
                I[c] = in;
                iv[c] = 1.0 / in;
            }
            /* every effective distance scaled by I_old/I_new >= mu */
            M = M * mu * (1.0 - 1e-15);
            E = E * mu * (1.0 + 1e-15);
            tsweep += omp_get_wtime() - t0;
        }
        inf.rounds += 1;
        inf.sweeps += sw;
        inf.balanced = balanced;

        /* new centers: compensated sums in input order (R9) */
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) Ain[perm[i]] = A[i];
        nsum* acc = (nsum*)calloc((size_t)k * (d + 1), sizeof(nsum));
        if (!acc) { rc = PC_ENOMEM; goto done; }
        for (int64_t i = 0; i < n; ++i) {
            int c = Ain[i];
            for (int j = 0; j < d; ++j) nsum_add(&acc[(int64_t)c * (d + 1) + j], X[j][i]);
            nsum_add(&acc[(int64_t)c * (d + 1) + d], 1.0);
        }
        double dmax = 0.0;
        for (int c = 0; c < k; ++c) {
            double w = acc[(int64_t)c * (d + 1) + d].s + acc[(int64_t)c * (d + 1) + d].c;
            for (int j = 0; j < d; ++j) {
                nsum* q = &acc[(int64_t)c * (d + 1) + j];
                double v = C[(int64_t)c * d + j];
                if (w > 0.0) v = (q->s + q->c) / w;
                Cn[(int64_t)c * d + j] = v;
            }
            double dx = Cn[(int64_t)c * d] - C[(int64_t)c * d];
            double dy = Cn[(int64_t)c * d + 1] - C[(int64_t)c * d + 1];
            double s = dx * dx + dy * dy;
            if (d == 3) {
                double dz = Cn[(int64_t)c * d + 2] - C[(int64_t)c * d + 2];
                s = s + dz * dz;
            }
            delta[c] = sqrt(s);
            if (delta[c] > dmax) dmax = delta[c];
        }
        free(acc);
        if (dmax < thr) {
            inf.converged = 1;
            memcpy(C, Cn, (size_t)k * d * sizeof(double));
            break;
        }
        double mu = 1.0, emax = 0.0;
        if (erosion) {
            /* beta: mean bounding-box diagonal of the non-empty blocks (R7) */
            double* bl = (double*)malloc((size_t)k * 2 * d * sizeof(double));
            if (!bl) { rc = PC_ENOMEM; goto done; }
            for (int c = 0; c < k; ++c)
                for (int j = 0; j < d; ++j) {
                    bl[(int64_t)c * 2 * d + j] = INFINITY;
                    bl[(int64_t)c * 2 * d + d + j] = -INFINITY;
                }
            for (int64_t i = 0; i < n; ++i) {
                double* q = bl + (int64_t)Ain[i] * 2 * d;
                for (int j = 0; j < d; ++j) {
                    q[j] = fmin(q[j], X[j][i]);
                    q[d + j] = fmax(q[d + j], X[j][i]);
                }
            }
            nsum bs = {0.0, 0.0};
            int64_t ne = 0;
            for (int c = 0; c < k; ++c) {
                if (cnt[c] == 0) continue;
                const double* q = bl + (int64_t)c * 2 * d;
                double ex = q[d] - q[0], ey = q[d + 1] - q[1];
                double s = ex * ex + ey * ey;
                if (d == 3) {
                    double ez = q[d + 2] - q[2];
                    s = s + ez * ez;
                }
                nsum_add(&bs, sqrt(s));
                ne += 1;
            }
            free(bl);
            const double beta = (bs.s + bs.c) / (double)ne;
            mu = INFINITY;
            for (int c = 0; c < k; ++c) {
                double io = I[c];
                if (delta[c] != 0.0) {
                    double t = -delta[c] / beta;
                    if (t > 0.0) t = 0.0;
                    double alpha = 2.0 / (1.0 + exp(t)) - 1.0;
                    I[c] = exp((1.0 - alpha) * log(I[c]));
                }
                iv[c] = 1.0 / I[c];
                mu = fmin(mu, io / I[c]);
            }
        }
        /* movement: upper bounds grow by the own center's movement (stored
         * relative to the accumulated movement), lower bounds shrink by the
         * largest movement over the influence (G1 relaxation) */
        for (int c = 0; c < k; ++c) {
            Dm[c] = (Dm[c] + delta[c]) * (1.0 + 1e-15);
            emax = fmax(emax, delta[c] * iv[c]);
        }
        M = M * mu * (1.0 - 1e-15);
        E = (E * mu + emax) * (1.0 + 1e-15);
        memcpy(C, Cn, (size_t)k * d * sizeof(double));
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) A_out[perm[i]] = A[i];
    if (centers_out) memcpy(centers_out, C, (size_t)k * d * sizeof(double));
    if (influence_out) memcpy(influence_out, I, (size_t)k * sizeof(double));
    inf.sweep_seconds = tsweep;
    inf.total_seconds = omp_get_wtime() - t_start;
    if (info) *info = inf;
done:
    free(ord); free(perm); free(xs[0]); free(xs[1]); free(xs[2]); free(A); free(Ain); free(ub);
    free(lb); free(tbox); free(sbox); free(slist); free(scnt); free(C); free(Cn); free(I); free(iv);
    free(Dm); free(delta); free(cnt); free(tcnt);
    return rc;
}

int pruned_num_threads(void) { return omp_get_max_threads(); }

void pruned_set_threads(int t)
{
    if (t > 0) omp_set_num_threads(t);
}
