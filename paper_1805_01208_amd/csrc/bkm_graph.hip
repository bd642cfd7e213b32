// Graph-quality evaluation (Sec. 2, the block measures; Sec. 5.2, Metrics):
// k-nearest-neighbour graphs of the point clouds, their undirected CSR form,
// and the edge cut, communication volume and block diameter bounds of a
// partition.
//
//   * k_knn: one wave per 64-point group of the Hilbert-ordered tiled layout.
//     Each lane keeps the K best (squared distance, input index) pairs of its
//     point in registers.  The wave first scans its own group and the two
//     curve neighbours, takes the largest K-th distance over its lanes as the
//     search radius, and then walks the hyper-tile / super-tile / tile /
//     group box hierarchy, visiting only groups whose box lies within the
//     radius (which shrinks as the lists fill).  Squared distances are FP64
//     ((dx*dx + dy*dy) + dz*dz, no contraction) and the box distance is the
//     same expression over per-axis gaps, so by monotone rounding a group
//     holding a point within the radius is never pruned: the lists are the
//     exact ones.
//   * symmetrisation: a directed entry p -> q that has no partner q -> p adds
//     p to q's row; rows are then sorted by index.
//   * metrics: one thread per vertex for cut and communication volume.  The
//     diameter bound (Sec. 5.2, Metrics: the first 3 rounds of iFUB, from a
//     4-sweep) runs every block at once: blocks are disjoint, so one
//     level-synchronous frontier serves them all.  The 4-sweep and the
//     search from its middle vertex u are five single-source searches per
//     block; a round's fringe (the vertices at distance i from u) is searched
//     bit-parallel, 64 sources per block and pass, each vertex holding a
//     64-bit mask of the sources that reached it, and the deepest level any
//     source reaches is the largest eccentricity of the fringe.
#include <climits>

#include <algorithm>

#include "bkm_internal.h"

namespace bkm {
namespace {

inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

__device__ inline double coord(const RunDev& r, int j, int64_t i)
{
    return r.in_f32 ? (double)r.xs32[j][i] : r.xs64[j][i];
}

// (da, ia) before (db, ib): smaller squared distance, then smaller index.
__device__ inline bool nb_before(double da, int32_t ia, double db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

template <int D>
__device__ inline double box_gap2(const double* a, const double* b)
{
    double g[D];
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = fmax(0.0, fmax(b[j] - a[D + j], a[j] - b[D + j]));
    double s = g[0] * g[0] + g[1] * g[1];
    if (D == 3) s = s + g[D - 1] * g[D - 1];
    return s;
}

__device__ inline double readlane_d(double v, int i)
{
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, i);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | lo);
}

template <int D, int K>
struct KnnLane {
    double q[D];
    int32_t self;
    bool active;
    double kd[K];
    int32_t ki[K];

    // All 64 points of group h against this lane's point.
    __device__ inline void visit(const RunDev& r, int64_t h, int lane)
    {
        const int64_t p2 = h * kWave + lane;
        const int32_t pid = r.perm[p2];
        double c[D];
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = coord(r, j, p2);
        for (int i = 0; i < kWave; ++i) {
            const int32_t pi = __builtin_amdgcn_readlane(pid, i);
            if (pi < 0) continue;   // padding (uniform)
            double dv[D];
#pragma unroll
            for (int j = 0; j < D; ++j) dv[j] = q[j] - readlane_d(c[j], i);
            double s = dv[0] * dv[0] + dv[1] * dv[1];
            if (D == 3) s = s + dv[D - 1] * dv[D - 1];
            if (active && pi != self && nb_before(s, pi, kd[K - 1], ki[K - 1])) {
                kd[K - 1] = s;
                ki[K - 1] = pi;
#pragma unroll
                for (int m = K - 1; m > 0; --m) {
                    if (nb_before(kd[m], ki[m], kd[m - 1], ki[m - 1])) {
                        const double td = kd[m];
                        kd[m] = kd[m - 1];
                        kd[m - 1] = td;
                        const int32_t ti = ki[m];
                        ki[m] = ki[m - 1];
                        ki[m - 1] = ti;
                    }
                }
            }
        }
    }

    // Search radius of the wave: the largest K-th squared distance of its
    // active lanes (infinite while some list is not full).
    __device__ inline double radius2() const { return wave_max_d(active ? kd[K - 1] : 0.0); }
};

template <int D, int K>
__global__ __launch_bounds__(kBlock) void k_knn(RunDev r, int32_t* nbr,
                                                unsigned long long* visits)
{
    const int lane = threadIdx.x % kWave;
    const int64_t g = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (g >= r.ngroups) return;
    KnnLane<D, K> L;
    const int64_t pos = g * kWave + lane;
    L.self = r.perm[pos];
    L.active = L.self >= 0;
    if (__ballot(L.active) == 0) return;   // a group of padding only
#pragma unroll
    for (int j = 0; j < D; ++j) L.q[j] = coord(r, j, pos);
#pragma unroll
    for (int m = 0; m < K; ++m) {
        L.kd[m] = INFINITY;
        L.ki[m] = INT_MAX;
    }
    double gb[2 * D];
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) gb[j] = r.gbox[g * 2 * D + j];

    long long nvis = 0;
    L.visit(r, g, lane);
    ++nvis;
    if (g > 0) {
        L.visit(r, g - 1, lane);
        ++nvis;
    }
    if (g + 1 < r.ngroups) {
        L.visit(r, g + 1, lane);
        ++nvis;
    }
    double R2 = L.radius2();

    const int gpt = r.T / kWave;   // groups per tile
    for (int hb = 0; hb < r.nhyper; hb += kWave) {
        const int h = hb + lane;
        const bool okh = h < r.nhyper && box_gap2<D>(gb, r.hbox + (int64_t)h * 2 * D) <= R2;
        unsigned long long mh = __ballot(okh);
        while (mh) {
            const int hi = hb + __builtin_ctzll(mh);
            mh &= mh - 1;
            const int s = hi * kHyper + lane;
            const bool oks = lane < kHyper && s < r.nsuper &&
                             box_gap2<D>(gb, r.sbox + (int64_t)s * 2 * D) <= R2;
            unsigned long long ms = __ballot(oks);
            while (ms) {
                const int si = hi * kHyper + __builtin_ctzll(ms);
                ms &= ms - 1;
                const int t = si * r.super_tiles + lane;
                const bool okt = lane < r.super_tiles && t < r.ntiles &&
                                 box_gap2<D>(gb, r.tbox + (int64_t)t * 2 * D) <= R2;
                unsigned long long mt = __ballot(okt);
                while (mt) {
                    const int ti = si * r.super_tiles + __builtin_ctzll(mt);
                    mt &= mt - 1;
                    const int64_t gg = (int64_t)ti * gpt + lane;
                    const bool okg = lane < gpt && gg < r.ngroups &&
                                     (gg < g - 1 || gg > g + 1) &&
                                     box_gap2<D>(gb, r.gbox + gg * 2 * D) <= R2;
                    unsigned long long mg = __ballot(okg);
                    while (mg) {
                        const int64_t gi = (int64_t)ti * gpt + __builtin_ctzll(mg);
                        mg &= mg - 1;
                        L.visit(r, gi, lane);
                        ++nvis;
                        R2 = L.radius2();
                    }
                }
            }
        }
    }
    if (L.active) {
#pragma unroll
        for (int m = 0; m < K; ++m) nbr[(int64_t)L.self * K + m] = L.ki[m];
    }
    if (lane == 0) atomicAdd(visits, (unsigned long long)nvis);
}

// ------------------------------------------------------------ symmetrise
// Directed entries p -> q (q = nbr[p][j]) without the partner q -> p: one
// more slot in q's row.  Out-of-range neighbours set *bad.
__global__ __launch_bounds__(kBlock) void k_sym_count(int64_t n, int K, const int32_t* nbr,
                                                      int32_t* extra, int* bad)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * K) return;
    const int64_t p = e / K;
    const int32_t q = nbr[e];
    if (q < 0 || q >= n || q == p) {
        atomicOr(bad, 1);
        return;
    }
    bool back = false;
    for (int i = 0; i < K; ++i) back |= nbr[(int64_t)q * K + i] == (int32_t)p;
    if (!back) atomicAdd(&extra[q], 1);
}

// Exclusive scan of the row lengths K + extra[p] into row_ptr (n + 1
// entries): per-block sums, a one-block scan of those, then the rows.
constexpr int kScanItems = 8;
constexpr int kScanBlock = 1024;
constexpr int kScanTile = kScanItems * kScanBlock;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* sh, int64_t* total)
{
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    int64_t x = v;
    for (int m = 1; m < kWave; m <<= 1) {
        const int64_t y = __shfl_up(x, m, kWave);
        if (lane >= m) x += y;
    }
    if (lane == kWave - 1) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int w = 0; w < kScanBlock / kWave; ++w) {
            const int64_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[kScanBlock / kWave] = run;
    }
    __syncthreads();
    const int64_t out = sh[wv] + x - v;
    if (total) *total = sh[kScanBlock / kWave];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(int64_t n, int K, const int32_t* extra,
                                                           int64_t* part)
{
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += K + extra[base + i];
    int64_t tot;
    block_exclusive_scan(s, sh, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_parts(int64_t nparts, int64_t* part)
{
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    int64_t carry = 0;
    for (int64_t base = 0; base < nparts; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nparts ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nparts) part[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_rows(int64_t n, int K, const int32_t* extra,
                                                          const int64_t* part, int64_t* row_ptr)
{
    __shared__ int64_t sh[kScanBlock / kWave + 1];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += K + extra[base + i];
    int64_t run = part[blockIdx.x] + block_exclusive_scan(s, sh, nullptr);
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) {
            row_ptr[base + i] = run;
            run += K + extra[base + i];
        }
        if (base + i == n) row_ptr[n] = run;
    }
}

__global__ __launch_bounds__(kBlock) void k_sym_fill(int64_t n, int K, const int32_t* nbr,
                                                     const int64_t* row_ptr, int32_t* cursor,
                                                     int32_t* col)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * K) return;
    const int64_t p = e / K;
    const int32_t q = nbr[e];
    col[row_ptr[p] + e % K] = q;
    bool back = false;
    for (int i = 0; i < K; ++i) back |= nbr[(int64_t)q * K + i] == (int32_t)p;
    if (!back) {
        const int slot = atomicAdd(&cursor[q], 1);
        col[row_ptr[q] + K + slot] = (int32_t)p;
    }
}

__global__ __launch_bounds__(kBlock) void k_sym_sort(int64_t n, const int64_t* row_ptr,
                                                     int32_t* col)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int64_t a = row_ptr[p], b = row_ptr[p + 1];
    for (int64_t i = a + 1; i < b; ++i) {
        const int32_t v = col[i];
        int64_t j = i;
        while (j > a && col[j - 1] > v) {
            col[j] = col[j - 1];
            --j;
        }
        col[j] = v;
    }
}

// --------------------------------------------------------------- metrics
// Per vertex: validation, cut entries, the number of other blocks among its
// neighbours (each counted at its first neighbour in that block), block size
// and lowest vertex.  Any out-of-range assignment, row pointer or column
// sets *bad and the vertex is skipped.
__global__ __launch_bounds__(kBlock) void k_gm_vertex(int64_t n, int64_t nnz, const int64_t* row_ptr,
                                                      const int32_t* col, const int32_t* A, int k,
                                                      GraphDev g)
{
    const int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    long long cut = 0;
    if (u < n) {
        const int32_t a = A[u];
        const int64_t rs = row_ptr[u], re = row_ptr[u + 1];
        bool ok = a >= 0 && a < k && rs >= 0 && rs <= re && re <= nnz;
        if (ok)
            for (int64_t e = rs; e < re; ++e) ok &= col[e] >= 0 && col[e] < n;
        if (!ok) {
            atomicOr(g.bad, 1);
        } else {
            long long vol = 0;
            for (int64_t e = rs; e < re; ++e) {
                const int32_t b = A[col[e]];
                if (b == a) continue;
                ++cut;
                bool dup = false;
                for (int64_t f = rs; f < e && !dup; ++f) dup = A[col[f]] == b;
                if (!dup) ++vol;
            }
            if (vol) atomicAdd((unsigned long long*)&g.comm[a], (unsigned long long)vol);
            atomicAdd(&g.size[a], 1);
            atomicMin(&g.seed[a], (int32_t)u);
        }
    }
    cut = wave_sum_ll(cut);
    if (threadIdx.x % kWave == 0 && cut) atomicAdd((unsigned long long*)g.cut2, (unsigned long long)cut);
}

__device__ inline unsigned long long far_key(int32_t level, int32_t v)
{
    return ((unsigned long long)(unsigned)level << 32) | (0xFFFFFFFFu - (unsigned)v);
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t* p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ULL;
}

__device__ inline int32_t far_vertex(unsigned long long key)
{
    return (int32_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
}

__device__ inline int32_t far_level(unsigned long long key) { return (int32_t)(key >> 32); }

// With dist from a search of block b whose far end x lies `steps` levels or
// more from its source: the vertex `steps` levels closer to the source on
// the path back from x, each step to the lowest-index neighbour of the
// block one level closer.
__device__ int32_t walk_back(const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                             const int32_t* dist, int32_t b, int32_t x, int32_t steps)
{
    for (int32_t t = 0; t < steps && x >= 0; ++t) {
        const int32_t want = dist[x] - 1;
        int32_t nx = -1;
        for (int64_t e = row_ptr[x]; e < row_ptr[(int64_t)x + 1]; ++e) {
            const int32_t y = col[e];
            if (A[y] == b && dist[y] == want && (nx < 0 || y < nx)) nx = y;
        }
        x = nx;
    }
    return x;
}

// Per-block bookkeeping between the single-source searches of the diameter
// bound, from the results of the search just finished (far, reached, dist):
//   stage 0: source r1 = the lowest vertex;
//   stage 1: connected iff the search reached the whole block; source a1;
//   stage 2: ecc(a1); source r2, floor(ecc/2) from a1 on the path from b1;
//   stage 3: source a2;
//   stage 4: l = max(ecc(a1), ecc(a2)); source u, floor(ecc/2) from a2 on
//            the path from b2;
//   stage 5: iFUB start from ecc(u): i, lb, ub; counts the blocks left open.
__global__ __launch_bounds__(kBlock) void k_diam_stage(int k, GraphDev g, int stage,
                                                       const int64_t* row_ptr, const int32_t* col,
                                                       const int32_t* A, const int32_t* dist)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= k) return;
    int32_t src = -1;
    const unsigned long long key = g.far[b];
    if (stage == 0) {
        g.conn[b] = 0;
        if (g.size[b] > 0) src = g.seed[b];
    } else if (stage == 1) {
        const int c = g.size[b] > 0 && g.reached[b] == g.size[b] ? 1 : 0;
        g.conn[b] = c;
        if (c) src = far_vertex(key);
    } else if (g.conn[b]) {
        const int32_t e = far_level(key);
        if (stage == 2) {
            g.ecc1[b] = e;
            src = walk_back(row_ptr, col, A, dist, b, far_vertex(key), e - e / 2);
        } else if (stage == 3) {
            src = far_vertex(key);
        } else if (stage == 4) {
            g.lval[b] = max(g.ecc1[b], e);
            src = walk_back(row_ptr, col, A, dist, b, far_vertex(key), e - e / 2);
        } else {
            g.fi[b] = e;
            g.lb[b] = max(g.lval[b], e);
            g.ub[b] = 2 * e;
            g.fcnt[b] = 0;
            g.blast[b] = -1;
            if (g.ub[b] > g.lb[b]) atomicAdd(&g.ctl[0], 1);
        }
    }
    g.src[b] = src;
}

// Seeds the next single-source search from g.src (resets every block's
// reached count and farthest vertex).
__global__ __launch_bounds__(kBlock) void k_bfs_sources(int k, GraphDev g, int32_t* dist,
                                                        int32_t* queue, int32_t* count)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= k) return;
    const int32_t src = g.src[b];
    g.reached[b] = 0;
    g.far[b] = 0;
    if (src < 0) return;
    dist[src] = 0;
    g.reached[b] = 1;
    g.far[b] = far_key(0, src);
    queue[atomicAdd(count, 1)] = src;
}

// iFUB round, fringe: every vertex of an open block at distance i from u
// gets its rank in the block's fringe (the order does not matter: a round
// takes the largest eccentricity over the whole fringe); the largest fringe
// goes to ctl[1].
__global__ __launch_bounds__(kBlock) void k_fringe_rank(int64_t n, const int32_t* A,
                                                        const int32_t* du, GraphDev g,
                                                        int32_t* frank)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const int32_t b = A[v];
    int32_t r = -1;
    if (g.conn[b] && g.ub[b] > g.lb[b] && du[v] == g.fi[b]) {
        r = atomicAdd(&g.fcnt[b], 1);
        atomicMax(&g.ctl[1], r + 1);
    }
    frank[v] = r;
}

// Sources of batch `batch`: fringe ranks 64*batch .. 64*batch + 63 of every
// block, each with its own bit.
__global__ __launch_bounds__(kBlock) void k_mbfs_seed(int64_t n, const int32_t* frank, int batch,
                                                      unsigned long long* arrive, int32_t* queue,
                                                      int32_t* count)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const int32_t r = v < n ? frank[v] - 64 * batch : -1;
    const bool src = r >= 0 && r < 64;
    if (src) arrive[v] = 1ULL << r;
    const unsigned long long b = __ballot(src);
    if (b == 0ULL) return;
    int base = 0;
    if (lane == __builtin_ctzll(b)) base = atomicAdd(count, (int)__popcll(b));
    base = __shfl(base, __builtin_ctzll(b), kWave);
    if (src) queue[base + (int)__popcll(b & ((1ULL << lane) - 1ULL))] = (int32_t)v;
}

// Round end: B = the deepest level the fringe's searches reached.  If
// max(lb, B) > 2(i - 1) the bound is exact (lb = ub), else lb = max(lb, B),
// ub = 2(i - 1) and the next round looks one level closer to u.
__global__ __launch_bounds__(kBlock) void k_ifub_round(int k, GraphDev g)
{
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= k || !g.conn[b] || g.ub[b] <= g.lb[b]) return;
    const int32_t i = g.fi[b];
    const int32_t m = max(g.lb[b], g.blast[b]);
    if (m > 2 * (i - 1)) {
        g.lb[b] = m;
        g.ub[b] = m;
    } else {
        g.lb[b] = m;
        g.ub[b] = 2 * (i - 1);
        g.fi[b] = i - 1;
    }
    g.fcnt[b] = 0;
    g.blast[b] = -1;
    if (g.ub[b] > g.lb[b]) atomicAdd(&g.ctl[0], 1);
}

// One level: every frontier vertex claims its unvisited neighbours of the
// same block; a claimed vertex joins the next frontier and may become its
// block's farthest vertex.  kBfsLanes lanes share a frontier vertex, each
// taking every kBfsLanes-th entry of its row; the lanes of a wave reserve
// their places in the next frontier with one atomic per step.
constexpr int kBfsLanes = 8;

// The frontier size comes from device memory (counts[level % 3]), so the
// host can enqueue many levels without reading it: a fixed grid walks the
// frontier, and a level whose frontier is empty does nothing.  The level
// adds to counts[(level + 1) % 3], which the level before cleared, and
// clears counts[(level + 2) % 3] for the level after; `levels` counts the
// levels with a non-empty frontier.
__global__ __launch_bounds__(kBlock) void k_bfs_level(const int64_t* row_ptr, const int32_t* col,
                                                      const int32_t* A, GraphDev g,
                                                      const int32_t* frontier, int32_t* counts,
                                                      int32_t level, int32_t* dist, int32_t* next,
                                                      int32_t* levels)
{
    const int32_t fcount = counts[level % 3];
    int32_t* ncount = counts + (level + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[(level + 2) % 3] = 0;
        if (fcount > 0) atomicAdd(levels, 1);
    }
    const int lane = threadIdx.x % kWave;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    const int64_t per_block = kBlock / kBfsLanes;
    // block-uniform walk over the frontier, kBlock / kBfsLanes vertices per block and step
    for (int64_t i0 = (int64_t)blockIdx.x * per_block; i0 < fcount;
         i0 += (int64_t)gridDim.x * per_block) {
        const int64_t i = i0 + threadIdx.x / kBfsLanes;
        const bool act = i < fcount;
        int32_t u = 0, a = -1;
        int64_t e = 0, end = 0;
        if (act) {
            u = frontier[i];
            a = A[u];
            e = row_ptr[u] + threadIdx.x % kBfsLanes;
            end = row_ptr[(int64_t)u + 1];
        }
        while (__ballot(e < end) != 0ULL) {
            bool claim = false;
            int32_t v = 0;
            if (e < end) {
                v = col[e];
                e += kBfsLanes;
                claim = A[v] == a && dist[v] == -1 && atomicCAS(&dist[v], -1, level + 1) == -1;
            }
            const unsigned long long b = __ballot(claim);
            if (b == 0ULL) continue;
            int base = 0;
            if (lane == __builtin_ctzll(b)) base = atomicAdd(ncount, (int)__popcll(b));
            base = __shfl(base, __builtin_ctzll(b), kWave);
            if (claim) next[base + (int)__popcll(b & below)] = v;
            // block counters: one update per distinct block among the claims
            unsigned long long pend = b;
            while (pend) {
                const int leader = __builtin_ctzll(pend);
                const int la = __shfl(a, leader, kWave);
                const bool mine = claim && a == la;
                const unsigned long long mm = __ballot(mine);
                unsigned long long key = mine ? far_key(level + 1, v) : 0ULL;
                for (int m = kWave / 2; m > 0; m >>= 1) {
                    const unsigned long long o = __shfl_xor(key, m, kWave);
                    key = o > key ? o : key;
                }
                if (lane == leader) {
                    atomicAdd(&g.reached[la], (int)__popcll(mm));
                    atomicMax(&g.far[la], key);
                }
                pend &= ~mm;
            }
        }
    }
}

// One level of the bit-parallel search: a frontier vertex takes the bits
// that first reached it at this level (its arrival mask minus the bits it
// has seen), records the level as its block's deepest, and offers them to
// its neighbours of the same block; a neighbour whose arrival mask for the
// next level was empty joins the next frontier.  A neighbour read while it
// is itself updating its seen mask may be offered bits it already has: it
// drops them at the next level, so every bit arrives at every vertex at its
// true distance from the source.  Frontier sizes rotate as in k_bfs_level.
__global__ __launch_bounds__(kBlock) void k_mbfs_level(const int64_t* row_ptr, const int32_t* col,
                                                       const int32_t* A, GraphDev g,
                                                       const int32_t* frontier, int32_t* counts,
                                                       int32_t level, unsigned long long* seen,
                                                       unsigned long long* cur,
                                                       unsigned long long* nxt, int32_t* next,
                                                       int32_t* levels)
{
    const int32_t fcount = counts[level % 3];
    int32_t* ncount = counts + (level + 1) % 3;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[(level + 2) % 3] = 0;
        if (fcount > 0) atomicAdd(levels, 1);
    }
    const int lane = threadIdx.x % kWave;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    const int64_t per_block = kBlock / kBfsLanes;
    for (int64_t i0 = (int64_t)blockIdx.x * per_block; i0 < fcount;
         i0 += (int64_t)gridDim.x * per_block) {
        const int64_t i = i0 + threadIdx.x / kBfsLanes;
        const bool act = i < fcount;
        int32_t u = 0, a = -1;
        int64_t e = 0, end = 0;
        unsigned long long m = 0ULL;
        if (act) {
            u = frontier[i];
            a = A[u];
            const unsigned long long sn = seen[u];
            m = cur[u] & ~sn;
            // the lanes of u's group all read cur and seen above (same wave)
            if (threadIdx.x % kBfsLanes == 0) {
                cur[u] = 0ULL;
                if (m) {
                    seen[u] = sn | m;
                    atomicMax(&g.blast[a], level);
                }
            }
            if (m) {
                e = row_ptr[u] + threadIdx.x % kBfsLanes;
                end = row_ptr[(int64_t)u + 1];
            }
        }
        while (__ballot(e < end) != 0ULL) {
            bool app = false;
            int32_t v = 0;
            if (e < end) {
                v = col[e];
                e += kBfsLanes;
                if (A[v] == a) {
                    const unsigned long long add = m & ~seen[v];
                    if (add) app = atomicOr(&nxt[v], add) == 0ULL;
                }
            }
            const unsigned long long b = __ballot(app);
            if (b == 0ULL) continue;
            int base = 0;
            if (lane == __builtin_ctzll(b)) base = atomicAdd(ncount, (int)__popcll(b));
            base = __shfl(base, __builtin_ctzll(b), kWave);
            if (app) next[base + (int)__popcll(b & below)] = v;
        }
    }
}

// Block results after the searches, and the summary (one block).
__global__ __launch_bounds__(1024) void k_gm_final(int k, GraphDev g, int32_t* diam_out,
                                                   int32_t* diam_ub_out, int64_t* comm_out,
                                                   double* summary)
{
    __shared__ double sh[1024 / kWave];
    __shared__ long long shl[3][1024 / kWave];
    long long mxc = 0, tot = 0, disc = 0;
    double mxd = 0.0, inv = 0.0, counted = 0.0, exact = 0.0;
    for (int b = threadIdx.x; b < k; b += 1024) {
        const long long c = g.comm[b];
        mxc = c > mxc ? c : mxc;
        tot += c;
        int32_t dm, du;
        if (g.size[b] == 0) {
            dm = du = 0;
        } else if (g.conn[b] == 0) {
            dm = du = -1;
            ++disc;
        } else {
            dm = g.lb[b];
            du = g.ub[b];
            if (dm == du) exact += 1.0;
        }
        if (diam_ub_out) diam_ub_out[b] = du;
        if (g.size[b] >= 2) {
            counted += 1.0;
            if (dm > 0) inv += 1.0 / (double)dm;
        }
        mxd = fmax(mxd, (double)dm);
        if (diam_out) diam_out[b] = dm;
        if (comm_out) comm_out[b] = c;
    }
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int m = kWave / 2; m > 0; m >>= 1) {
        const long long o = __shfl_xor(mxc, m, kWave);
        mxc = o > mxc ? o : mxc;
    }
    tot = wave_sum_ll(tot);
    disc = wave_sum_ll(disc);
    if (lane == 0) {
        shl[0][wv] = mxc;
        shl[1][wv] = tot;
        shl[2][wv] = disc;
    }
    mxd = wave_max_d(mxd);
    inv = wave_sum_d(inv);
    counted = wave_sum_d(counted);
    exact = wave_sum_d(exact);
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0, t = 0, dsc = 0;
        for (int w = 0; w < 1024 / kWave; ++w) {
            a = shl[0][w] > a ? shl[0][w] : a;
            t += shl[1][w];
            dsc += shl[2][w];
        }
        summary[0] = (double)a;
        summary[1] = (double)t;
        summary[2] = (double)dsc;
        g.sums[0] = a;
        g.sums[1] = t;
        g.sums[2] = dsc;
    }
    if (lane == 0) sh[wv] = mxd;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) m = fmax(m, sh[w]);
        summary[3] = m;
    }
    __syncthreads();
    if (lane == 0) sh[wv] = inv;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) s += sh[w];
        summary[4] = s;
    }
    __syncthreads();
    if (lane == 0) sh[wv] = counted;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) s += sh[w];
        summary[5] = s;
    }
    __syncthreads();
    if (lane == 0) sh[wv] = exact;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 1024 / kWave; ++w) s += sh[w];
        summary[6] = s;
    }
}

template <int D>
hipError_t launch_knn_d(const RunDev& r, int K, int32_t* nbr, unsigned long long* visits,
                        hipStream_t s)
{
    const unsigned grid = nblocks(r.ngroups, kBlock / kWave);
    switch (K) {
#define BKM_KNN_CASE(KK) \
    case KK: k_knn<D, KK><<<grid, kBlock, 0, s>>>(r, nbr, visits); break;
        BKM_KNN_CASE(1) BKM_KNN_CASE(2) BKM_KNN_CASE(3) BKM_KNN_CASE(4)
        BKM_KNN_CASE(5) BKM_KNN_CASE(6) BKM_KNN_CASE(7) BKM_KNN_CASE(8)
        BKM_KNN_CASE(9) BKM_KNN_CASE(10) BKM_KNN_CASE(11) BKM_KNN_CASE(12)
        BKM_KNN_CASE(13) BKM_KNN_CASE(14) BKM_KNN_CASE(15) BKM_KNN_CASE(16)
#undef BKM_KNN_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_knn(const RunDev& r, int K, int32_t* nbr, unsigned long long* visits,
                      hipStream_t s)
{
    return r.d == 2 ? launch_knn_d<2>(r, K, nbr, visits, s) : launch_knn_d<3>(r, K, nbr, visits, s);
}

hipError_t launch_sym_count(int64_t n, int K, const int32_t* nbr, int32_t* extra, int* bad,
                            hipStream_t s)
{
    k_sym_count<<<nblocks(n * K, kBlock), kBlock, 0, s>>>(n, K, nbr, extra, bad);
    return hipGetLastError();
}

int64_t scan_parts(int64_t n) { return (n + 1 + kScanTile - 1) / kScanTile; }

hipError_t launch_sym_rows(int64_t n, int K, const int32_t* extra, int64_t* part,
                           int64_t* row_ptr, hipStream_t s)
{
    // n + 1 row pointers: the tiles cover indices 0..n
    const int64_t np = scan_parts(n);
    k_scan_tiles<<<(unsigned)np, kScanBlock, 0, s>>>(n, K, extra, part);
    k_scan_parts<<<1, kScanBlock, 0, s>>>(np, part);
    k_scan_rows<<<(unsigned)np, kScanBlock, 0, s>>>(n, K, extra, part, row_ptr);
    return hipGetLastError();
}

hipError_t launch_sym_fill(int64_t n, int K, const int32_t* nbr, const int64_t* row_ptr,
                           int32_t* cursor, int32_t* col, hipStream_t s)
{
    k_sym_fill<<<nblocks(n * K, kBlock), kBlock, 0, s>>>(n, K, nbr, row_ptr, cursor, col);
    k_sym_sort<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, row_ptr, col);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s)
{
    if (n > 0) k_fill_i32<<<nblocks(n, kBlock), kBlock, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_gm_vertex(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                            const int32_t* A, int k, const GraphDev& g, hipStream_t s)
{
    k_gm_vertex<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, nnz, row_ptr, col, A, k, g);
    return hipGetLastError();
}

hipError_t launch_diam_stage(int k, const GraphDev& g, int stage, const int64_t* row_ptr,
                             const int32_t* col, const int32_t* A, const int32_t* dist,
                             hipStream_t s)
{
    k_diam_stage<<<nblocks(k, kBlock), kBlock, 0, s>>>(k, g, stage, row_ptr, col, A, dist);
    return hipGetLastError();
}

hipError_t launch_bfs_sources(int k, const GraphDev& g, int32_t* dist, int32_t* queue,
                              int32_t* count, hipStream_t s)
{
    k_bfs_sources<<<nblocks(k, kBlock), kBlock, 0, s>>>(k, g, dist, queue, count);
    return hipGetLastError();
}

hipError_t launch_fringe_rank(int64_t n, const int32_t* A, const int32_t* du, const GraphDev& g,
                              int32_t* frank, hipStream_t s)
{
    k_fringe_rank<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, A, du, g, frank);
    return hipGetLastError();
}

hipError_t launch_mbfs_seed(int64_t n, const int32_t* frank, int batch,
                            unsigned long long* arrive, int32_t* queue, int32_t* count,
                            hipStream_t s)
{
    k_mbfs_seed<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, frank, batch, arrive, queue, count);
    return hipGetLastError();
}

hipError_t launch_mbfs_level(const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                             const GraphDev& g, const int32_t* frontier, int32_t* counts,
                             int32_t level, unsigned long long* seen, unsigned long long* cur,
                             unsigned long long* nxt, int32_t* next, int32_t* levels, int64_t n,
                             hipStream_t s)
{
    const unsigned grid = (unsigned)std::min<int64_t>(2048, nblocks(n * kBfsLanes, kBlock));
    k_mbfs_level<<<grid, kBlock, 0, s>>>(row_ptr, col, A, g, frontier, counts, level, seen, cur,
                                         nxt, next, levels);
    return hipGetLastError();
}

hipError_t launch_ifub_round(int k, const GraphDev& g, hipStream_t s)
{
    k_ifub_round<<<nblocks(k, kBlock), kBlock, 0, s>>>(k, g);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s)
{
    if (n > 0) k_fill_u64<<<nblocks(n, kBlock), kBlock, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const int64_t* row_ptr, const int32_t* col, const int32_t* A,
                            const GraphDev& g, const int32_t* frontier, int32_t* counts,
                            int32_t level, int32_t* dist, int32_t* next, int32_t* levels,
                            int64_t n, hipStream_t s)
{
    // enough blocks for a frontier of n vertices in one step, at most 2048
    const unsigned grid = (unsigned)std::min<int64_t>(2048, nblocks(n * kBfsLanes, kBlock));
    k_bfs_level<<<grid, kBlock, 0, s>>>(row_ptr, col, A, g, frontier, counts, level, dist, next,
                                        levels);
    return hipGetLastError();
}

hipError_t launch_gm_final(int k, const GraphDev& g, int32_t* diam_out, int32_t* diam_ub_out,
                           int64_t* comm_out, double* summary, hipStream_t s)
{
    k_gm_final<<<1, 1024, 0, s>>>(k, g, diam_out, diam_ub_out, comm_out, summary);
    return hipGetLastError();
}

}  // namespace bkm
