/*
 * Graph-quality evaluation oracle: plain, slow, obviously correct FP64 / integer
 * CPU code.  TEST INFRASTRUCTURE ONLY: nothing in the product path may call it.
 *
 * The paper judges partitions on the meshes' graphs (Sec. 2, the block
 * measures; Sec. 5.2, Metrics): edge cut, maximum and total communication
 * volume, and a lower bound on each block's diameter.  Its meshes are not
 * available, so the graphs here are k-nearest-neighbour graphs of the point
 * clouds, made undirected.
 *
 * Readings taken where the paper is silent or inconsistent:
 *   K1  knn(p) = the K points q != p with the smallest (squared Euclidean
 *       distance ((dx*dx + dy*dy) + dz*dz), index of q), in that order.
 *   K2  The graph has the edge {p, q} when q is in knn(p) or p in knn(q);
 *       it is stored as CSR with both directions, rows sorted ascending.
 *   M1  Edge cut = number of undirected edges whose ends lie in different
 *       blocks (Sec. 2).
 *   M2  comm(V_i) = sum over v in V_i of the number of blocks other than
 *       V_i holding a neighbour of v.  The printed formula does not exclude
 *       V_i, but the paper's tables report a total volume below the edge
 *       cut, which only the reading without V_i allows.
 *   M3  The diameter is bounded from below as in Sec. 5.2 (a lower bound
 *       within a factor 2 of the exact value, from breadth-first searches):
 *       a double sweep inside the block's induced subgraph, from the block's
 *       vertex of lowest index to the farthest vertex found (largest hop
 *       distance, lowest index on ties), whose eccentricity is the bound.
 *       A block that this search does not cover is disconnected and has
 *       diameter infinity (reported as -1); an empty block reports 0.
 *   M4  The diameters are aggregated by their harmonic mean (Sec. 5.3), over
 *       the blocks of at least two vertices, with 1/infinity = 0; it is
 *       infinity when all of them are disconnected and 0 when there are
 *       none.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)
#define KNN_MAX 64

/* Squared distance of points i and j, evaluated in the written order. */
static double sq_dist(int d, const double* const* X, int64_t i, int64_t j)
{
    double dx = X[0][i] - X[0][j];
    double dy = X[1][i] - X[1][j];
    double s = dx * dx + dy * dy;
    if (d == 3) {
        double dz = X[2][i] - X[2][j];
        s = s + dz * dz;
    }
    return s;
}

/* (da, ia) before (db, ib): smaller distance, then smaller index (K1). */
static int nb_before(double da, int32_t ia, double db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* K nearest neighbours of the points queries[0..nq) by brute force over all
 * n points (reading K1).  nbr is [nq][K], input indices, nearest first. */
int oracle_knn_of(int64_t n, int d, const double* const* X, int K, int64_t nq,
                  const int64_t* queries, int32_t* nbr)
{
    if (n < 2 || n > INT32_MAX || d < 2 || d > 3 || K < 1 || K > KNN_MAX || K > n - 1)
        return ORC_EINVAL;
    for (int64_t t = 0; t < nq; ++t)
        if (queries[t] < 0 || queries[t] >= n) return ORC_EINVAL;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nq; ++t) {
        const int64_t i = queries[t];
        double bd[KNN_MAX];
        int32_t bi[KNN_MAX];
        for (int m = 0; m < K; ++m) {
            bd[m] = INFINITY;
            bi[m] = INT32_MAX;
        }
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double s = sq_dist(d, X, i, j);
            if (!nb_before(s, (int32_t)j, bd[K - 1], bi[K - 1])) continue;
            int m = K - 1;
            while (m > 0 && nb_before(s, (int32_t)j, bd[m - 1], bi[m - 1])) {
                bd[m] = bd[m - 1];
                bi[m] = bi[m - 1];
                --m;
            }
            bd[m] = s;
            bi[m] = (int32_t)j;
        }
        memcpy(nbr + t * K, bi, (size_t)K * sizeof(int32_t));
    }
    return ORC_OK;
}

/* K nearest neighbours of every point (reading K1): nbr is [n][K]. */
int oracle_knn(int64_t n, int d, const double* const* X, int K, int32_t* nbr)
{
    if (n < 2 || n > INT32_MAX) return ORC_EINVAL;
    int64_t* all = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!all) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) all[i] = i;
    int rc = oracle_knn_of(n, d, X, K, n, all, nbr);
    free(all);
    return rc;
}

static int cmp_pair(const void* a, const void* b)
{
    const int64_t* x = (const int64_t*)a;
    const int64_t* y = (const int64_t*)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

/* Undirected graph of the neighbour lists (reading K2): every (p, q) and
 * (q, p) pair, sorted, duplicates dropped, as CSR.  row_ptr has n+1
 * entries; col needs room for 2*n*K.  *nnz receives the stored entries. */
int oracle_knn_symmetrize(int64_t n, int K, const int32_t* nbr, int64_t* row_ptr,
                          int32_t* col, int64_t* nnz)
{
    if (n < 1 || K < 1) return ORC_EINVAL;
    int64_t m = 2 * n * (int64_t)K;
    int64_t* pairs = (int64_t*)malloc((size_t)m * 2 * sizeof(int64_t));
    if (!pairs) return ORC_ENOMEM;
    int64_t e = 0;
    for (int64_t p = 0; p < n; ++p)
        for (int j = 0; j < K; ++j) {
            int64_t q = nbr[p * K + j];
            if (q < 0 || q >= n) { free(pairs); return ORC_EINVAL; }
            pairs[2 * e] = p; pairs[2 * e + 1] = q; ++e;
            pairs[2 * e] = q; pairs[2 * e + 1] = p; ++e;
        }
    qsort(pairs, (size_t)m, 2 * sizeof(int64_t), cmp_pair);
    int64_t out = 0;
    for (int64_t p = 0; p <= n; ++p) row_ptr[p] = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i > 0 && pairs[2 * i] == pairs[2 * i - 2] && pairs[2 * i + 1] == pairs[2 * i - 1])
            continue;
        col[out++] = (int32_t)pairs[2 * i + 1];
        row_ptr[pairs[2 * i] + 1] += 1;
    }
    for (int64_t p = 0; p < n; ++p) row_ptr[p + 1] += row_ptr[p];
    *nnz = out;
    free(pairs);
    return ORC_OK;
}

typedef struct {
    int64_t edge_cut;
    int64_t max_comm;
    int64_t total_comm;
    int32_t max_diameter;          /* largest finite block diameter bound */
    int32_t disconnected_blocks;
    double harmonic_diameter;      /* reading M4 */
} oracle_graph_stats;

/* Breadth-first search from src inside block b (vertices with A == b);
 * dist (n entries, -1 = unreached) is written for the block's vertices.
 * Returns the number of vertices reached; *far receives the farthest one
 * (largest distance, lowest index) and *ecc its distance. */
static int64_t block_bfs(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                         int32_t b, int64_t src, int32_t* dist, int64_t* queue, int64_t* far,
                         int32_t* ecc)
{
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    *far = src;
    *ecc = 0;
    while (head < tail) {
        int64_t u = queue[head++];
        if (dist[u] > *ecc || (dist[u] == *ecc && u < *far)) {
            *ecc = dist[u];
            *far = u;
        }
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t v = col[e];
            if (A[v] != b || dist[v] >= 0) continue;
            dist[v] = dist[u] + 1;
            queue[tail++] = v;
        }
    }
    (void)n;
    return tail;
}

/* Edge cut, communication volumes and diameter bounds of the partition A of
 * the CSR graph (readings M1-M4).  comm ([k]) and diam ([k]) may be NULL. */
int oracle_graph_metrics(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                         int k, int64_t* comm_out, int32_t* diam_out, oracle_graph_stats* st)
{
    if (n < 1 || k < 1 || !st) return ORC_EINVAL;
    for (int64_t u = 0; u < n; ++u) {
        if (A[u] < 0 || A[u] >= k) return ORC_EINVAL;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (col[e] < 0 || col[e] >= n) return ORC_EINVAL;
    }
    int64_t* comm = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int32_t* diam = (int32_t*)calloc((size_t)k, sizeof(int32_t));
    int64_t* size = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int64_t* seed = (int64_t*)malloc((size_t)k * sizeof(int64_t));
    int32_t* dist = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int64_t* queue = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int rc = ORC_OK;
    if (!comm || !diam || !size || !seed || !dist || !queue) { rc = ORC_ENOMEM; goto done; }

    int64_t cut2 = 0;   /* directed cut entries: each undirected edge twice */
    for (int b = 0; b < k; ++b) seed[b] = -1;
    for (int64_t u = 0; u < n; ++u) {
        int32_t a = A[u];
        size[a] += 1;
        if (seed[a] < 0) seed[a] = u;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int32_t b = A[col[e]];
            if (b == a) continue;
            cut2 += 1;
            /* block b counts once for vertex u: at its first neighbour in b */
            int dup = 0;
            for (int64_t f = row_ptr[u]; f < e; ++f)
                if (A[col[f]] == b) { dup = 1; break; }
            if (!dup) comm[a] += 1;
        }
    }
    st->edge_cut = cut2 / 2;
    st->max_comm = 0;
    st->total_comm = 0;
    for (int b = 0; b < k; ++b) {
        st->total_comm += comm[b];
        if (comm[b] > st->max_comm) st->max_comm = comm[b];
    }

    for (int64_t u = 0; u < n; ++u) dist[u] = -1;
    st->max_diameter = 0;
    st->disconnected_blocks = 0;
    double inv = 0.0;
    int counted = 0;
    for (int b = 0; b < k; ++b) {
        if (size[b] == 0) { diam[b] = 0; continue; }
        int64_t far;
        int32_t ecc;
        int64_t reached = block_bfs(n, row_ptr, col, A, b, seed[b], dist, queue, &far, &ecc);
        if (reached < size[b]) {
            diam[b] = -1;
            st->disconnected_blocks += 1;
        } else {
            for (int64_t i = 0; i < reached; ++i) dist[queue[i]] = -1;
            int64_t far2;
            block_bfs(n, row_ptr, col, A, b, far, dist, queue, &far2, &ecc);
            diam[b] = ecc;
            if (ecc > st->max_diameter) st->max_diameter = ecc;
        }
        if (size[b] >= 2) {
            counted += 1;
            if (diam[b] > 0) inv += 1.0 / (double)diam[b];
        }
    }
    if (counted == 0) st->harmonic_diameter = 0.0;
    else if (inv == 0.0) st->harmonic_diameter = INFINITY;
    else st->harmonic_diameter = (double)counted / inv;
    if (comm_out) memcpy(comm_out, comm, (size_t)k * sizeof(int64_t));
    if (diam_out) memcpy(diam_out, diam, (size_t)k * sizeof(int32_t));
done:
    free(comm); free(diam); free(size); free(seed); free(dist); free(queue);
    return rc;
}
