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
 *   M3  The diameter of a block is bounded from below as in Sec. 5.2: by the
 *       first 3 rounds of the iFUB algorithm (Crescenzi, Grossi, Habib,
 *       Lanzi, Marino, Theor. Comput. Sci. 514, 2013) in the block's induced
 *       subgraph, started from a 4-sweep of the same paper:
 *         r1 = the block's lowest vertex, a1 = farthest from r1, b1 =
 *         farthest from a1, r2 = the vertex at distance floor(ecc(a1)/2)
 *         from a1 on an a1-b1 path; a2 = farthest from r2, b2 = farthest
 *         from a2, u = the vertex at distance floor(ecc(a2)/2) from a2 on an
 *         a2-b2 path; l = max(ecc(a1), ecc(a2)).  "Farthest" is the largest
 *         hop distance, lowest index on ties; the path runs back from b to
 *         the source, each step to the lowest-index neighbour one level
 *         closer to it.
 *         iFUB from u: i = ecc(u), lb = max(l, i), ub = 2i.  A round, taken
 *         while ub > lb and at most 3 times: B = the largest eccentricity of
 *         the vertices at distance i from u; if max(lb, B) > 2(i-1) then
 *         lb = ub = max(lb, B) (exact); else lb = max(lb, B), ub = 2(i-1),
 *         i = i-1.
 *       The bound is lb (<= diameter <= ub; exact when lb == ub).  A block
 *       that the search from r1 does not cover is disconnected and has
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
    int32_t exact_blocks;          /* non-empty connected blocks with lb == ub (M3) */
    double harmonic_diameter;      /* reading M4 */
} oracle_graph_stats;

/* The induced subgraph of one block: its vertices in ascending order
 * (local index = position) and, for every vertex, its neighbours in the
 * block as local indices (ascending, since CSR rows are sorted and the local
 * order follows the global one). */
typedef struct {
    int64_t m;           /* vertices */
    const int64_t* v;    /* global ids, ascending */
    int64_t* rp;         /* [m+1] local row pointers */
    int64_t* ci;         /* local column indices */
} block_graph;

/* Breadth-first search from local vertex src: dist[m] (-1 = unreached) is
 * written; returns the number of vertices reached; *far receives the
 * farthest one (largest distance, lowest index) and *ecc its distance. */
static int64_t bfs_local(const block_graph* g, int64_t src, int32_t* dist, int64_t* queue,
                         int64_t* far, int32_t* ecc)
{
    for (int64_t x = 0; x < g->m; ++x) dist[x] = -1;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    *far = src;
    *ecc = 0;
    while (head < tail) {
        int64_t x = queue[head++];
        if (dist[x] > *ecc || (dist[x] == *ecc && x < *far)) {
            *ecc = dist[x];
            *far = x;
        }
        for (int64_t e = g->rp[x]; e < g->rp[x + 1]; ++e) {
            int64_t y = g->ci[e];
            if (dist[y] >= 0) continue;
            dist[y] = dist[x] + 1;
            queue[tail++] = y;
        }
    }
    return tail;
}

/* With dist from a search whose source lies at distance D from b: the vertex
 * at distance D - steps from the source on the path from b back towards it,
 * each step to the lowest-index neighbour one level closer. */
static int64_t walk_back(const block_graph* g, const int32_t* dist, int64_t b, int32_t steps)
{
    int64_t x = b;
    for (int32_t t = 0; t < steps; ++t) {
        int64_t nx = -1;
        for (int64_t e = g->rp[x]; e < g->rp[x + 1]; ++e) {
            int64_t y = g->ci[e];
            if (dist[y] == dist[x] - 1 && (nx < 0 || y < nx)) nx = y;
        }
        x = nx;
    }
    return x;
}

/* Diameter bound of one connected block (reading M3); *ub_out receives the
 * proven upper bound.  trace (NULL or 10 entries) receives, as local
 * indices and values: a1, b1, r2, a2, b2, u, l, rounds taken, lb, ub. */
static int32_t block_ifub(const block_graph* g, int32_t* dist, int32_t* du, int64_t* queue,
                          int32_t* ub_out, int64_t* trace)
{
    int64_t far;
    int32_t ecc;
    /* 4-sweep */
    bfs_local(g, 0, dist, queue, &far, &ecc);                 /* r1 = lowest vertex */
    const int64_t a1 = far;
    bfs_local(g, a1, dist, queue, &far, &ecc);
    const int64_t b1 = far;
    const int32_t ecc_a1 = ecc;
    const int64_t r2 = walk_back(g, dist, far, ecc_a1 - ecc_a1 / 2);
    bfs_local(g, r2, dist, queue, &far, &ecc);
    const int64_t a2 = far;
    bfs_local(g, a2, dist, queue, &far, &ecc);
    const int64_t b2 = far;
    const int32_t ecc_a2 = ecc;
    const int64_t u = walk_back(g, dist, far, ecc_a2 - ecc_a2 / 2);
    const int32_t l = ecc_a1 > ecc_a2 ? ecc_a1 : ecc_a2;
    /* iFUB from u, first 3 rounds */
    bfs_local(g, u, du, queue, &far, &ecc);
    int32_t i = ecc;
    int32_t lb = l > ecc ? l : ecc;
    int32_t ub = 2 * ecc;
    int round = 0;
    for (; round < 3 && ub > lb; ++round) {
        int32_t B = 0;
        for (int64_t x = 0; x < g->m; ++x) {
            if (du[x] != i) continue;
            int64_t fx;
            int32_t ex;
            bfs_local(g, x, dist, queue, &fx, &ex);
            if (ex > B) B = ex;
        }
        const int32_t m = lb > B ? lb : B;
        if (m > 2 * (i - 1)) {
            lb = ub = m;
        } else {
            lb = m;
            ub = 2 * (i - 1);
            i -= 1;
        }
    }
    *ub_out = ub;
    if (trace) {
        const int64_t t[10] = {a1, b1, r2, a2, b2, u, l, round, lb, ub};
        memcpy(trace, t, sizeof(t));
    }
    return lb;
}

/* Edge cut, communication volumes and diameter bounds of the partition A of
 * the CSR graph (readings M1-M4).  comm, diam and diam_ub ([k]) may be NULL;
 * diam_ub receives the proven upper bounds (-1 disconnected, 0 empty). */
int oracle_graph_metrics(int64_t n, const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                         int k, int64_t* comm_out, int32_t* diam_out, int32_t* diam_ub_out,
                         oracle_graph_stats* st)
{
    if (n < 1 || k < 1 || !st) return ORC_EINVAL;
    for (int64_t u = 0; u < n; ++u) {
        if (A[u] < 0 || A[u] >= k) return ORC_EINVAL;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e)
            if (col[e] < 0 || col[e] >= n) return ORC_EINVAL;
    }
    int64_t* comm = (int64_t*)calloc((size_t)k, sizeof(int64_t));
    int32_t* diam = (int32_t*)calloc((size_t)k, sizeof(int32_t));
    int32_t* dub = (int32_t*)calloc((size_t)k, sizeof(int32_t));
    int64_t* start = (int64_t*)calloc((size_t)k + 1, sizeof(int64_t));
    int64_t* verts = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* loc = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int rc = ORC_OK;
    if (!comm || !diam || !dub || !start || !verts || !loc) { rc = ORC_ENOMEM; goto done; }

    int64_t cut2 = 0;   /* directed cut entries: each undirected edge twice */
    for (int64_t u = 0; u < n; ++u) {
        int32_t a = A[u];
        start[a + 1] += 1;
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

    /* the vertices of every block, ascending; local index of every vertex */
    for (int b = 0; b < k; ++b) start[b + 1] += start[b];
    {
        int64_t* fill = (int64_t*)malloc((size_t)k * sizeof(int64_t));
        if (!fill) { rc = ORC_ENOMEM; goto done; }
        memcpy(fill, start, (size_t)k * sizeof(int64_t));
        for (int64_t u = 0; u < n; ++u) {
            loc[u] = fill[A[u]] - start[A[u]];
            verts[fill[A[u]]++] = u;
        }
        free(fill);
    }

    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : fail)
    for (int b = 0; b < k; ++b) {
        const int64_t m = start[b + 1] - start[b];
        if (m == 0) { diam[b] = 0; dub[b] = 0; continue; }
        block_graph g;
        g.m = m;
        g.v = verts + start[b];
        int64_t nnz = 0;
        for (int64_t x = 0; x < m; ++x)
            for (int64_t e = row_ptr[g.v[x]]; e < row_ptr[g.v[x] + 1]; ++e)
                nnz += A[col[e]] == b;
        g.rp = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
        g.ci = (int64_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
        int32_t* dist = (int32_t*)malloc((size_t)m * sizeof(int32_t));
        int32_t* du = (int32_t*)malloc((size_t)m * sizeof(int32_t));
        int64_t* queue = (int64_t*)malloc((size_t)m * sizeof(int64_t));
        if (!g.rp || !g.ci || !dist || !du || !queue) {
            fail = 1;
        } else {
            int64_t t = 0;
            for (int64_t x = 0; x < m; ++x) {
                g.rp[x] = t;
                for (int64_t e = row_ptr[g.v[x]]; e < row_ptr[g.v[x] + 1]; ++e)
                    if (A[col[e]] == b) g.ci[t++] = loc[col[e]];
            }
            g.rp[m] = t;
            int64_t far;
            int32_t ecc;
            if (bfs_local(&g, 0, dist, queue, &far, &ecc) < m) {
                diam[b] = -1;
                dub[b] = -1;
            } else {
                diam[b] = block_ifub(&g, dist, du, queue, &dub[b], NULL);
            }
        }
        free(g.rp); free(g.ci); free(dist); free(du); free(queue);
    }
    if (fail) { rc = ORC_ENOMEM; goto done; }

    st->max_diameter = 0;
    st->disconnected_blocks = 0;
    st->exact_blocks = 0;
    double inv = 0.0;
    int counted = 0;
    for (int b = 0; b < k; ++b) {
        const int64_t m = start[b + 1] - start[b];
        if (m == 0) continue;
        if (diam[b] < 0) {
            st->disconnected_blocks += 1;
        } else {
            if (diam[b] > st->max_diameter) st->max_diameter = diam[b];
            if (diam[b] == dub[b]) st->exact_blocks += 1;
        }
        if (m >= 2) {
            counted += 1;
            if (diam[b] > 0) inv += 1.0 / (double)diam[b];
        }
    }
    if (counted == 0) st->harmonic_diameter = 0.0;
    else if (inv == 0.0) st->harmonic_diameter = INFINITY;
    else st->harmonic_diameter = (double)counted / inv;
    if (comm_out) memcpy(comm_out, comm, (size_t)k * sizeof(int64_t));
    if (diam_out) memcpy(diam_out, diam, (size_t)k * sizeof(int32_t));
    if (diam_ub_out) memcpy(diam_ub_out, dub, (size_t)k * sizeof(int32_t));
done:
    free(comm); free(diam); free(dub); free(start); free(verts); free(loc);
    return rc;
}

/* The steps of reading M3 on a whole connected graph taken as one block:
 * trace[10] = a1, b1, r2, a2, b2, u, l, rounds taken, lb, ub (vertex ids;
 * r1 is vertex 0).  Returns ORC_EINVAL when the graph is not connected. */
int oracle_ifub_trace(int64_t n, const int64_t* row_ptr, const int32_t* col, int64_t* trace)
{
    if (n < 1 || !trace) return ORC_EINVAL;
    block_graph g;
    int64_t* ids = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* ci = (int64_t*)malloc((size_t)(row_ptr[n] > 0 ? row_ptr[n] : 1) * sizeof(int64_t));
    int64_t* rp = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t* dist = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int32_t* du = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    int64_t* queue = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int rc = ORC_OK;
    if (!ids || !ci || !rp || !dist || !du || !queue) { rc = ORC_ENOMEM; goto out; }
    for (int64_t x = 0; x < n; ++x) ids[x] = x;
    for (int64_t x = 0; x <= n; ++x) rp[x] = row_ptr[x];
    for (int64_t e = 0; e < row_ptr[n]; ++e) {
        if (col[e] < 0 || col[e] >= n) { rc = ORC_EINVAL; goto out; }
        ci[e] = col[e];
    }
    g.m = n;
    g.v = ids;
    g.rp = rp;
    g.ci = ci;
    int64_t far;
    int32_t ecc, ub;
    if (bfs_local(&g, 0, dist, queue, &far, &ecc) < n) { rc = ORC_EINVAL; goto out; }
    block_ifub(&g, dist, du, queue, &ub, trace);
out:
    free(ids); free(ci); free(rp); free(dist); free(du); free(queue);
    return rc;
}
