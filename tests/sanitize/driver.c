/*
 * Sanitizer driver for the host C code of the tests and measurements: the
 * oracle (oracle/*.c) and the pruned CPU baseline (baseline/pruned_cpu.c)
 * are compiled with AddressSanitizer and UndefinedBehaviorSanitizer together
 * with this file, which calls every exported function on small random and
 * degenerate inputs.  Any out-of-bounds access, leak or undefined operation
 * aborts the program with a report.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t rounds, sweeps, balanced, converged; double imbalance, mbw, lmax; } oinfo;
typedef struct { double imbalance, objective, lmax; int32_t empty, over; } ostats;
typedef struct { int64_t cut, mxc, totc; int32_t mxd, disc, exact; double harm; } ogstats;
typedef struct { int32_t r, s, b, c; int64_t e, sk, ce; double t1, t2; } pinfo;

int oracle_bbox(int64_t, int, const double* const*, double*, double*);
uint64_t oracle_hilbert_index(const uint32_t*, int, int);
int oracle_sfc_keys(int64_t, int, const double* const*, int, uint64_t*);
int oracle_sfc_order(int64_t, const uint64_t*, int64_t*);
int oracle_init_centers_sfc(int64_t, int, const double* const*, int, int, const double*, double*,
                            int64_t*, uint64_t*);
int oracle_assign(int64_t, int, const double* const*, int, const double*, const double*, int32_t*,
                  double*, double*);
int oracle_block_weights(int64_t, const int32_t*, const double*, int, double*);
double oracle_total_weight(int64_t, const double*);
double oracle_lmax(int64_t, int, double, double, int);
int oracle_balance_step(int, int, const double*, double, double, double*);
int oracle_new_centers(int64_t, int, const double* const*, const double*, const int32_t*, int,
                       const double*, double*, double*);
double oracle_beta(int64_t, int, const double* const*, const int32_t*, int);
void oracle_erode(int, const double*, double, double*);
int oracle_balanced_kmeans(int64_t, int, const double* const*, const double*, int, double, int, int,
                           double, int, int, const double*, const double*, const double*, int32_t*,
                           double*, double*, double*, int32_t*, oinfo*);
int oracle_balanced_kmeans_sampled(int64_t, int, const double* const*, const double*, int, double,
                                   int, int, double, int, int, int64_t, const uint64_t*,
                                   const double*, int32_t*, double*, double*, double*, int32_t*,
                                   oinfo*, int32_t*, int32_t*);
int oracle_partition_stats(int64_t, int, const double* const*, const double*, const int32_t*, int,
                           double, const double*, double*, double*, ostats*);
int oracle_knn(int64_t, int, const double* const*, int, int32_t*);
int oracle_knn_symmetrize(int64_t, int, const int32_t*, int64_t*, int32_t*, int64_t*);
int oracle_graph_metrics(int64_t, const int64_t*, const int32_t*, const int32_t*, int, int64_t*,
                         int32_t*, int32_t*, ogstats*);
int oracle_ifub_trace(int64_t, const int64_t*, const int32_t*, int64_t*);
int pruned_balanced_kmeans(int64_t, int, const double* const*, int, double, int, int, double, int,
                           const double*, int32_t*, double*, double*, pinfo*);

static uint64_t rng_state = 88172645463325252ULL;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * 0x1p-53;
}

#define CHECK(x)                                                            \
    do {                                                                    \
        if ((x) < 0) {                                                      \
            fprintf(stderr, "call failed at line %d: %s\n", __LINE__, #x); \
            return 1;                                                       \
        }                                                                   \
    } while (0)

static int one_case(int64_t n, int d, int k, int weighted, int K)
{
    double* xs[3] = {0, 0, 0};
    for (int j = 0; j < d; ++j) {
        xs[j] = malloc((size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; ++i) xs[j][i] = urand() * (j + 1);
    }
    const double* const* X = (const double* const*)xs;
    double* W = NULL;
    if (weighted) {
        W = malloc((size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; ++i) W[i] = 0.5 + urand();
    }
    double lo[3], hi[3];
    CHECK(oracle_bbox(n, d, X, lo, hi));
    uint32_t q[3] = {3, 1, 2};
    (void)oracle_hilbert_index(q, d, 4);
    uint64_t* keys = malloc((size_t)n * sizeof(uint64_t));
    int64_t* perm = malloc((size_t)n * sizeof(int64_t));
    CHECK(oracle_sfc_keys(n, d, X, 16, keys));
    CHECK(oracle_sfc_order(n, keys, perm));
    double* C = malloc((size_t)k * d * sizeof(double));
    double* Cn = malloc((size_t)k * d * sizeof(double));
    double* I = malloc((size_t)k * sizeof(double));
    double* sz = malloc((size_t)k * sizeof(double));
    double* delta = malloc((size_t)k * sizeof(double));
    double* ts = malloc((size_t)k * sizeof(double));
    for (int c = 0; c < k; ++c) {
        I[c] = 0.9 + 0.2 * urand();
        ts[c] = 0.5 + urand();
    }
    CHECK(oracle_init_centers_sfc(n, d, X, k, 16, NULL, C, perm, keys));
    CHECK(oracle_init_centers_sfc(n, d, X, k, 16, ts, C, NULL, NULL));
    int32_t* A = malloc((size_t)n * sizeof(int32_t));
    double* best = malloc((size_t)n * sizeof(double));
    double* second = malloc((size_t)n * sizeof(double));
    CHECK(oracle_assign(n, d, X, k, C, I, A, best, second));
    CHECK(oracle_block_weights(n, A, W, k, sz));
    double tw = oracle_total_weight(n, W);
    double lmax = oracle_lmax(n, k, 0.03, tw, W == NULL);
    (void)oracle_balance_step(k, d, sz, lmax, tw / k, I);
    CHECK(oracle_new_centers(n, d, X, W, A, k, C, Cn, delta));
    double beta = oracle_beta(n, d, X, A, k);
    oracle_erode(k, delta, beta, I);
    oinfo inf;
    int32_t* spr = malloc(8 * sizeof(int32_t));
    CHECK(oracle_balanced_kmeans(n, d, X, W, k, 0.03, 8, 10, -1.0, 16, 1, NULL, NULL, NULL, A, Cn,
                                 I, sz, spr, &inf));
    CHECK(oracle_balanced_kmeans(n, d, X, W, k, 0.02, 8, 10, 0.0, 12, 0, NULL, NULL, ts, A, Cn,
                                 I, sz, spr, &inf));
    int32_t sr = 0, ss = 0;
    CHECK(oracle_balanced_kmeans_sampled(n, d, X, W, k, 0.03, 8, 10, -1.0, 16, 1, 3, keys, NULL,
                                         A, Cn, I, sz, spr, &inf, &sr, &ss));
    ostats st;
    CHECK(oracle_partition_stats(n, d, X, W, A, k, 0.03, ts, sz, Cn, &st));
    if (n > K) {
        int32_t* nbr = malloc((size_t)n * K * sizeof(int32_t));
        int64_t* rp = malloc((size_t)(n + 1) * sizeof(int64_t));
        int32_t* col = malloc((size_t)n * K * 2 * sizeof(int32_t));
        int64_t nnz = 0;
        CHECK(oracle_knn(n, d, X, K, nbr));
        CHECK(oracle_knn_symmetrize(n, K, nbr, rp, col, &nnz));
        int64_t* comm = malloc((size_t)k * sizeof(int64_t));
        int32_t* dm = malloc((size_t)k * sizeof(int32_t));
        int32_t* du = malloc((size_t)k * sizeof(int32_t));
        ogstats gs;
        CHECK(oracle_graph_metrics(n, rp, col, A, k, comm, dm, du, &gs));
        int64_t tr[10];
        (void)oracle_ifub_trace(n, rp, col, tr);   /* EINVAL when the graph is disconnected */
        free(nbr); free(rp); free(col); free(comm); free(dm); free(du);
    }
    if (!weighted) {
        pinfo pi;
        CHECK(oracle_init_centers_sfc(n, d, X, k, 16, NULL, C, NULL, NULL));
        CHECK(pruned_balanced_kmeans(n, d, X, k, 0.03, 8, 10, -1.0, 1, C, A, Cn, I, &pi));
        CHECK(pruned_balanced_kmeans(n, d, X, k, 0.03, 8, 10, -1.0, 0, C, A, Cn, I, &pi));
    }
    for (int j = 0; j < d; ++j) free(xs[j]);
    free(W); free(keys); free(perm); free(C); free(Cn); free(I); free(sz); free(delta); free(ts);
    free(A); free(best); free(second); free(spr);
    return 0;
}

int main(void)
{
    const int64_t ns[] = {1, 2, 7, 300, 2500};
    const int ks[] = {1, 2, 5, 17, 40};
    for (int t = 0; t < 5; ++t)
        for (int d = 2; d <= 3; ++d)
            for (int w = 0; w < 2; ++w) {
                int k = ks[t] < ns[t] ? ks[t] : (int)ns[t];
                if (one_case(ns[t], d, k, w, 4)) return 1;
            }
    printf("sanitized run ok\n");
    return 0;
}
