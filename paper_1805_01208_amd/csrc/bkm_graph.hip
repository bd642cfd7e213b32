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
//     group box hierarchy, visiting only boxes within the radius (which
//     shrinks as the lists fill); within a tile the test goes down to 8-point
//     parts of the groups, each with its own box.  A visited part's points
//     are the same for every lane: they arrive by scalar loads and enter the
//     arithmetic as SGPR operands.  Four partners at a time are screened with
//     a fused squared distance against a slightly widened K-th distance; the
//     wave computes exact distances and inserts only when a lane passes.
//     Exact squared distances are FP64 ((dx*dx + dy*dy) + dz*dz, no
//     contraction) and the box distance is the same expression over per-axis
//     gaps, so by monotone rounding a box holding a point within the radius
//     is never pruned: the lists are the exact ones.
//   * symmetrisation: a directed entry p -> q that has no partner q -> p adds
//     p to q's row; rows are then sorted by index.
//   * metrics: one thread per vertex for cut and communication volume.  The
//     diameter bound (Sec. 5.2, Metrics: the first 3 rounds of iFUB, from a
//     4-sweep) takes one workgroup per block: every block's first search in
//     one launch on the input graph, the other searches of the connected
//     blocks in a second, on their induced subgraphs relabelled so that
//     their data is contiguous.
//     The 4-sweep and the search from its middle vertex u are five
//     single-source searches; a round's fringe (the vertices at distance i
//     from u) is searched bit-parallel, 64 sources per pass, each vertex
//     holding a 64-bit mask of the sources that reached it, and the deepest
//     level any source reaches is the largest eccentricity of the fringe.
#include <climits>

#include <algorithm>

#include "bkm_graph_internal.h"
#include "bkm_internal.h"

namespace bkm {
namespace {

inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// (da, ia) before (db, ib): smaller squared distance, then smaller index
// (bitwise operators: the compiler keeps this free of branches).
__device__ inline bool nb_before(double da, int32_t ia, double db, int32_t ib)
{
    return (da < db) | ((da == db) & (ia < ib));
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

// Scalar (wave-uniform) loads: the partner points of a visited group are the
// same for every lane, so they are read through the scalar cache into SGPRs
// and enter the distance arithmetic as scalar operands.
typedef const __attribute__((address_space(4))) double* ScalarD;
typedef const __attribute__((address_space(4))) int32_t* ScalarI;

constexpr int kKnnChunk = 4;   // partners screened per wave-wide test
constexpr int kKnnSub = kWave / kKnnParts;   // points per part of a group

template <int D, int K>
struct KnnLane {
    double q[D];
    int32_t self;
    bool active;
    double kd[K];
    int32_t ki[K];

    // Screening radius of the lane: its K-th squared distance (infinite while
    // the list is not full), below zero for a padding lane.
    __device__ inline double limit() const { return active ? kd[K - 1] : -1.0; }

    // Insertion into the sorted list: the new pair replaces the K-th entry
    // and moves up while it comes before its upper neighbour; the wave stops
    // as soon as no lane moves (late insertions land near the end).
    __device__ inline void insert(double s, int32_t pi)
    {
        kd[K - 1] = s;
        ki[K - 1] = pi;
#pragma unroll
        for (int m = K - 1; m > 0; --m) {
            const bool c = nb_before(kd[m], ki[m], kd[m - 1], ki[m - 1]);
            if (__ballot(c) == 0ULL) break;
            const double td = kd[m - 1];
            const int32_t ti = ki[m - 1];
            kd[m - 1] = c ? kd[m] : td;
            ki[m - 1] = c ? ki[m] : ti;
            kd[m] = c ? td : kd[m];
            ki[m] = c ? ti : ki[m];
        }
    }

    // Screening limit: the limit widened by 2^-50 relative and 2^-1060
    // absolute.  The screen's fused squared distance and the exact one
    // ((dx*dx + dy*dy) + dz*dz) are both within a few units of 2^-53 of the
    // true sum of the same squares, so a pair within the limit by the exact
    // distance always passes the widened screen.
    __device__ inline double screen_limit() const
    {
        const double l = limit();
        return fma(fabs(l), 0x1p-50, l) + 0x1p-1060;
    }

    // Exact squared distance to partner slot i of the layout.
    __device__ inline double dist2(const double* const* x, int64_t i) const
    {
        double dv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) dv[j] = q[j] - ((ScalarD)x[j])[i];
        double d2 = dv[0] * dv[0] + dv[1] * dv[1];
        if (D == 3) d2 = d2 + dv[D - 1] * dv[D - 1];
        return d2;
    }

    // Points c0 .. c1 - 1 of group h (all 64 by default) against this lane's
    // point.  Four partners at a time are screened by a fused squared distance against the lane's
    // widened limit; only when some lane passes does the wave compute the
    // exact distances, test (squared distance, index) against the K-th entry
    // and insert.  A partner failing the screen fails the exact test too:
    // the limit only shrinks.  Padding slots hold copies of a real point and
    // are dropped by their index (-1).
    __device__ inline void visit(const double* const* x, const int32_t* perm, int64_t h, int c0 = 0,
                                 int c1 = kWave)
    {
        const int64_t base = h * kWave;
        double lim = screen_limit();
        for (int c = c0; c < c1; c += kKnnChunk) {
            unsigned long long hit = 0;
#pragma unroll
            for (int u = 0; u < kKnnChunk; ++u) {
                double dv[D];
#pragma unroll
                for (int j = 0; j < D; ++j) dv[j] = q[j] - ((ScalarD)x[j])[base + c + u];
                double d2 = dv[0] * dv[0];
#pragma unroll
                for (int j = 1; j < D; ++j) d2 = fma(dv[j], dv[j], d2);
                hit |= __ballot(d2 <= lim);
            }
            if (hit == 0) continue;
            int32_t ids[kKnnChunk];
#pragma unroll
            for (int u = 0; u < kKnnChunk; ++u) ids[u] = ((ScalarI)perm)[base + c + u];
#pragma unroll
            for (int u = 0; u < kKnnChunk; ++u) {
                const int32_t pi = ids[u];
                const double e = dist2(x, base + c + u);
                if (active && pi >= 0 && pi != self && nb_before(e, pi, kd[K - 1], ki[K - 1]))
                    insert(e, pi);
            }
            lim = screen_limit();
        }
    }

    // Search radius of the wave: the largest K-th squared distance of its
    // active lanes (infinite while some list is not full).
    __device__ inline double radius2() const { return wave_max_d(active ? kd[K - 1] : 0.0); }
};

// Boxes of the 8-point parts of every group (the search prunes at that
// granularity): one wave per group, min and max over each part.
template <int D>
__global__ __launch_bounds__(kBlock) void k_knn_partbox(RunDev r, KnnPts P, double* hb)
{
    const int lane = threadIdx.x % kWave;
    const int64_t g = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (g >= r.ngroups) return;
    double mn[D], mx[D];
#pragma unroll
    for (int j = 0; j < D; ++j) mn[j] = mx[j] = P.x[j][g * kWave + lane];
    for (int o = kKnnSub / 2; o > 0; o >>= 1) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            mn[j] = fmin(mn[j], __shfl_xor(mn[j], o, kWave));
            mx[j] = fmax(mx[j], __shfl_xor(mx[j], o, kWave));
        }
    }
    if (lane % kKnnSub == 0) {
        double* out = hb + (g * kKnnParts + lane / kKnnSub) * 2 * D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            out[j] = mn[j];
            out[D + j] = mx[j];
        }
    }
}

// FP64 copy of an FP32 layout (axis j at x + j * npad) for the search.
__global__ __launch_bounds__(kBlock) void k_knn_widen(RunDev r, double* x)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= r.npad) return;
    for (int j = 0; j < r.d; ++j) x[j * r.npad + p] = (double)r.xs32[j][p];
}

template <int D, int K>
__global__ __launch_bounds__(kBlock) void k_knn(RunDev r, KnnPts P, int32_t* nbr,
                                                unsigned long long* visits)
{
    const int lane = threadIdx.x % kWave;
    // wave-uniform group index: the group's box and the walk live in SGPRs
    const int64_t g = (int64_t)blockIdx.x * (kBlock / kWave) +
                      __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (g >= r.ngroups) return;
    KnnLane<D, K> L;
    const int64_t pos = g * kWave + lane;
    L.self = r.perm[pos];
    L.active = L.self >= 0;
    if (__ballot(L.active) == 0) return;   // a group of padding only
#pragma unroll
    for (int j = 0; j < D; ++j) L.q[j] = P.x[j][pos];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        L.kd[m] = INFINITY;
        L.ki[m] = INT_MAX;
    }
    double gb[2 * D];
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) gb[j] = r.gbox[g * 2 * D + j];

    long long nvis = 0;   // in 8-point parts
    L.visit(P.x, r.perm, g);
    nvis += kKnnParts;
    if (g > 0) {
        L.visit(P.x, r.perm, g - 1);
        nvis += kKnnParts;
    }
    if (g + 1 < r.ngroups) {
        L.visit(P.x, r.perm, g + 1);
        nvis += kKnnParts;
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
                    // the tile's 8-point parts within the radius (one lane
                    // each: at most 64 per tile), then the radius again
                    const int64_t hg = (int64_t)ti * gpt * kKnnParts + lane;
                    const int64_t gg = hg / kKnnParts;
                    const bool okg = lane < kKnnParts * gpt && gg < r.ngroups &&
                                     (gg < g - 1 || gg > g + 1) &&
                                     box_gap2<D>(gb, P.pbox + hg * 2 * D) <= R2;
                    unsigned long long mg = __ballot(okg);
                    while (mg) {
                        const int64_t hi = (int64_t)ti * gpt * kKnnParts + __builtin_ctzll(mg);
                        mg &= mg - 1;
                        const int c0 = (int)(hi % kKnnParts) * kKnnSub;
                        L.visit(P.x, r.perm, hi / kKnnParts, c0, c0 + kKnnSub);
                        ++nvis;
                    }
                    R2 = L.radius2();
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
// The entry passes take their vertices in a caller's order when one is given
// (a permutation of 0..n-1, e.g. the Hilbert order of the search): vertex t
// of the pass is order[t].  The results do not depend on it.  Each row is
// read again by every vertex that lists it; in a spatially coherent order
// those vertices come close together in time, so the rereads hit in cache.
__device__ inline int64_t vertex_at(const int32_t* order, int64_t t)
{
    return order ? (int64_t)order[t] : t;
}

// The order is a permutation of 0..n-1: every value in range (mark[v] = 1,
// mark zeroed before), then every mark set (and cleared again).
__global__ __launch_bounds__(kBlock) void k_order_mark(int64_t n, const int32_t* order,
                                                       int32_t* mark, int* bad)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n) return;
    const int32_t v = order[t];
    if (v < 0 || v >= n) atomicOr(bad, 1);
    else mark[v] = 1;
}

__global__ __launch_bounds__(kBlock) void k_order_check(int64_t n, int32_t* mark, int* bad)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    if (mark[v] != 1) atomicOr(bad, 1);
    mark[v] = 0;
}

// Directed entries p -> q (q = nbr[p][j]) without the partner q -> p: one
// more slot in q's row, and bit e of `miss` set (e = the entry's index in
// the pass, one 64-bit word per wave).  Out-of-range neighbours set *bad.
__global__ __launch_bounds__(kBlock) void k_sym_count(int64_t n, int K, const int32_t* nbr,
                                                      const int32_t* order, int32_t* extra,
                                                      unsigned long long* miss, int* bad)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool missing = false;
    if (e < n * K) {
        const int64_t p = vertex_at(order, e / K);
        const int32_t q = nbr[p * K + e % K];
        if (q < 0 || q >= n || q == p) {
            atomicOr(bad, 1);
        } else {
            bool back = false;
            for (int i = 0; i < K; ++i) back |= nbr[(int64_t)q * K + i] == (int32_t)p;
            if (!back) {
                atomicAdd(&extra[q], 1);
                missing = true;
            }
        }
    }
    const unsigned long long b = __ballot(missing);
    if (threadIdx.x % kWave == 0 && e < n * K) miss[e / kWave] = b;
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

// The lists themselves at the head of their rows, in input order (the
// reads and writes of neighbouring threads are adjacent).
__global__ __launch_bounds__(kBlock) void k_sym_copy(int64_t n, int K, const int32_t* nbr,
                                                     const int64_t* row_ptr, int32_t* col)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * K) return;
    col[row_ptr[e / K] + e % K] = nbr[e];
}

// The missing partners (bit e of `miss`, in the counting pass's order): p
// into q's row after its own list.
__global__ __launch_bounds__(kBlock) void k_sym_fill(int64_t n, int K, const int32_t* nbr,
                                                     const int32_t* order,
                                                     const unsigned long long* miss,
                                                     const int64_t* row_ptr, int32_t* cursor,
                                                     int32_t* col)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * K || !((miss[e / kWave] >> (e % kWave)) & 1ULL)) return;
    const int64_t p = vertex_at(order, e / K);
    const int32_t q = nbr[p * K + e % K];
    const int slot = atomicAdd(&cursor[q], 1);
    col[row_ptr[q] + K + slot] = (int32_t)p;
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
            int32_t own = 0;
            for (int64_t e = rs; e < re; ++e) {
                const int32_t b = A[col[e]];
                if (b == a) {
                    ++own;
                    continue;
                }
                ++cut;
                bool dup = false;
                for (int64_t f = rs; f < e && !dup; ++f) dup = A[col[f]] == b;
                if (!dup) ++vol;
            }
            g.ldeg[u] = own;
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

__device__ inline int32_t far_vertex(unsigned long long key)
{
    return (int32_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
}

__device__ inline int32_t far_level(unsigned long long key) { return (int32_t)(key >> 32); }

// With dist from a search whose far end x (a local id) lies `steps` levels
// or more from its source: the vertex `steps` levels closer to the source
// on the path back from x, each step to the neighbour one level closer with
// the lowest input index.
__device__ int32_t walk_back(const GraphDev& g, const int32_t* dist, int32_t x, int32_t steps)
{
    for (int32_t t = 0; t < steps && x >= 0; ++t) {
        const int32_t want = dist[x] - 1;
        int32_t nx = -1, nin = INT32_MAX;
        for (int64_t e = g.lrp[x]; e < g.lrp[(int64_t)x + 1]; ++e) {
            const int32_t y = g.lcol[e];
            if (dist[y] == want && g.mem[y] < nin) {
                nx = y;
                nin = g.mem[y];
            }
        }
        x = nx;
    }
    return x;
}

// ------------------------------------------------------ block diameters
// The diameter bound of a block (reading M3) lives in the block's induced
// subgraph, so one workgroup takes one block and runs all of its searches:
// the 4-sweep, the search from its middle vertex u, and up to three iFUB
// rounds.  Levels are separated by workgroup barriers only: a search of any
// length is part of one launch, and blocks proceed independently.
// After the first search, the connected blocks' induced subgraphs are
// relabelled block by block: local id = position in the block lists (mem),
// so block b holds the local ids moff[b] .. moff[b] + size - 1, and its rows
// (lrp, lcol) hold only its own edges.  Every array the later searches
// touch is then contiguous per block (distances, masks, queues, rows),
// instead of spread over the input order.  Ties still go by input index
// (mem of a local id).

constexpr int kBfsLanes = 8;   // lanes sharing a frontier vertex
constexpr int kDiamU = 4;      // frontier vertices a lane group holds at once

struct DiamShared {
    int cnt[2];                 // frontier sizes, alternating with the level
    int reached;                // vertices the search reached
    int levels;                 // levels with a non-empty frontier, over all searches
    int blast;                  // deepest level at which a fringe search reached a vertex
    int fcount;                 // fringe size
    int src;                    // a vertex chosen by thread 0
    unsigned long long far;     // far_key of the farthest vertex reached
};

// The graph a search walks.  InputView: the input graph restricted to block
// b (vertices by input index; a neighbour counts when it lies in b; the
// block's vertices listed in mem at off).  LocalView: a relabelled block
// (vertices by local id off .. off + size - 1; rows hold only own edges).
struct InputView {
    const int64_t* rp;
    const int32_t* col;
    const int32_t* A;
    const int32_t* mem;
    int32_t b;
    __device__ int32_t vertex(int32_t off, int32_t j) const { return mem[off + j]; }
    __device__ bool own(int32_t v) const { return A[v] == b; }
    __device__ int32_t input(int32_t v) const { return v; }
};
struct LocalView {
    const int64_t* rp;
    const int32_t* col;
    const int32_t* mem;
    __device__ int32_t vertex(int32_t off, int32_t j) const { return off + j; }
    __device__ bool own(int32_t) const { return true; }
    __device__ int32_t input(int32_t v) const { return mem[v]; }
};

// Single-source search of a block (off, size: its place in the block lists)
// from src, distances into d (every other vertex of the block at -1 first);
// leaves the reached count and the farthest vertex (largest level, lowest
// input index) in sh.  kBfsLanes lanes
// share a frontier vertex, each taking every kBfsLanes-th entry of its row,
// and every lane group holds kDiamU frontier vertices at once so that their
// loads overlap; a vertex is claimed by a CAS on its distance, and a wave
// reserves its claims' places in the next frontier with one LDS atomic.
template <int NT, typename View>
__device__ void bfs_block(const View& gv, int32_t off, int32_t size, int32_t src, int32_t* d,
                          int32_t* qa, int32_t* qb, DiamShared& sh)
{
    const int64_t* __restrict__ row_ptr = gv.rp;
    const int32_t* __restrict__ col = gv.col;
    constexpr int kPer = NT / kBfsLanes;
    const int tid = threadIdx.x, lane = tid % kWave;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int j = tid; j < size; j += NT) d[gv.vertex(off, j)] = -1;
    __syncthreads();
    if (tid == 0) {
        d[src] = 0;
        qa[0] = src;
        sh.cnt[0] = 1;
        sh.cnt[1] = 0;
        sh.reached = 1;
        sh.far = far_key(0, gv.input(src));
    }
    __syncthreads();
    int32_t* cur = qa;
    int32_t* nxt = qb;
    for (int level = 0;; ++level) {
        const int ncur = sh.cnt[level & 1];
        if (ncur == 0) break;
        int* ncount = &sh.cnt[(level + 1) & 1];
        for (int base = 0; base < ncur; base += kPer * kDiamU) {
            int64_t e[kDiamU], end[kDiamU];
#pragma unroll
            for (int q = 0; q < kDiamU; ++q) {
                const int i = base + q * kPer + tid / kBfsLanes;
                e[q] = end[q] = 0;
                if (i < ncur) {
                    const int32_t u = cur[i];
                    e[q] = row_ptr[u] + tid % kBfsLanes;
                    end[q] = row_ptr[(int64_t)u + 1];
                }
            }
            for (;;) {
                bool more = false;
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) more |= e[q] < end[q];
                if (__ballot(more) == 0ULL) break;
                int32_t v[kDiamU];
                bool live[kDiamU], claim[kDiamU];
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) {
                    live[q] = e[q] < end[q];
                    v[q] = live[q] ? col[e[q]] : 0;
                    e[q] += live[q] ? kBfsLanes : 0;
                }
#pragma unroll
                for (int q = 0; q < kDiamU; ++q)
                    claim[q] = live[q] && gv.own(v[q]) && d[v[q]] == -1;
#pragma unroll
                for (int q = 0; q < kDiamU; ++q)
                    if (claim[q]) claim[q] = atomicCAS(&d[v[q]], -1, level + 1) == -1;
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) {
                    const unsigned long long bm = __ballot(claim[q]);
                    if (bm == 0ULL) continue;
                    const int leader = __builtin_ctzll(bm);
                    int pos = 0;
                    if (lane == leader) {
                        pos = atomicAdd(ncount, (int)__popcll(bm));
                        atomicAdd(&sh.reached, (int)__popcll(bm));
                    }
                    pos = __shfl(pos, leader, kWave);
                    if (claim[q]) {
                        nxt[pos + (int)__popcll(bm & below)] = v[q];
                        atomicMax(&sh.far, far_key(level + 1, gv.input(v[q])));
                    }
                }
            }
        }
        __syncthreads();   // the next frontier is complete
        if (tid == 0) {
            sh.cnt[level & 1] = 0;   // the level after next appends here
            sh.levels += 1;
        }
        __syncthreads();
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
}

// Searches from up to 64 sources of the block at once (an iFUB round's fringe,
// source j with bit j): a vertex holds the sources that reached it (seen)
// and those arriving at the current level (arr[level & 1]); it joins the next
// frontier when the first new bit arrives.  sh.blast = the deepest level at
// which some vertex took a new bit, the largest eccentricity of the sources.
template <int NT>
__device__ void mbfs_block(const GraphDev& g, int32_t off, int32_t size, const int32_t* srcs,
                           int nsrc, unsigned long long* seen, unsigned long long* arr0,
                           unsigned long long* arr1, int32_t* qa, int32_t* qb, DiamShared& sh)
{
    const int64_t* __restrict__ row_ptr = g.lrp;
    const int32_t* __restrict__ col = g.lcol;
    constexpr int kPer = NT / kBfsLanes;
    const int tid = threadIdx.x, lane = tid % kWave;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int j = tid; j < size; j += NT) {
        const int32_t v = off + j;
        seen[v] = 0ULL;
        arr0[v] = 0ULL;
        arr1[v] = 0ULL;
    }
    __syncthreads();
    if (tid < nsrc) {
        const int32_t v = srcs[tid];
        arr0[v] = 1ULL << tid;
        qa[tid] = v;
    }
    if (tid == 0) {
        sh.cnt[0] = nsrc;
        sh.cnt[1] = 0;
        sh.blast = -1;
    }
    __syncthreads();
    int32_t* cur = qa;
    int32_t* nxt = qb;
    for (int level = 0;; ++level) {
        const int ncur = sh.cnt[level & 1];
        if (ncur == 0) break;
        int* ncount = &sh.cnt[(level + 1) & 1];
        unsigned long long* ca = (level & 1) ? arr1 : arr0;
        unsigned long long* na = (level & 1) ? arr0 : arr1;
        for (int base = 0; base < ncur; base += kPer * kDiamU) {
            int64_t e[kDiamU], end[kDiamU];
            unsigned long long m[kDiamU];
#pragma unroll
            for (int q = 0; q < kDiamU; ++q) {
                const int i = base + q * kPer + tid / kBfsLanes;
                e[q] = end[q] = 0;
                m[q] = 0ULL;
                if (i < ncur) {
                    const int32_t u = cur[i];
                    const unsigned long long sn = seen[u];
                    m[q] = ca[u] & ~sn;
                    // the lanes of u's group all read ca and seen above (same wave)
                    if (tid % kBfsLanes == 0) {
                        ca[u] = 0ULL;
                        if (m[q]) {
                            seen[u] = sn | m[q];
                            atomicMax(&sh.blast, level);
                        }
                    }
                    if (m[q]) {
                        e[q] = row_ptr[u] + tid % kBfsLanes;
                        end[q] = row_ptr[(int64_t)u + 1];
                    }
                }
            }
            for (;;) {
                bool more = false;
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) more |= e[q] < end[q];
                if (__ballot(more) == 0ULL) break;
                int32_t v[kDiamU];
                bool app[kDiamU];
                unsigned long long add[kDiamU];
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) {
                    const bool live = e[q] < end[q];
                    v[q] = live ? col[e[q]] : 0;
                    e[q] += live ? kBfsLanes : 0;
                    add[q] = live ? m[q] : 0ULL;
                }
#pragma unroll
                for (int q = 0; q < kDiamU; ++q)
                    if (add[q]) add[q] &= ~seen[v[q]];
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) app[q] = add[q] && atomicOr(&na[v[q]], add[q]) == 0ULL;
#pragma unroll
                for (int q = 0; q < kDiamU; ++q) {
                    const unsigned long long bm = __ballot(app[q]);
                    if (bm == 0ULL) continue;
                    const int leader = __builtin_ctzll(bm);
                    int pos = 0;
                    if (lane == leader) pos = atomicAdd(ncount, (int)__popcll(bm));
                    pos = __shfl(pos, leader, kWave);
                    if (app[q]) nxt[pos + (int)__popcll(bm & below)] = v[q];
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            sh.cnt[level & 1] = 0;
            sh.levels += 1;
        }
        __syncthreads();
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
}

// Diameter bounds, one block per workgroup (reading M3):
//   r1 = the lowest vertex; connected iff its search reaches the whole block;
//   a1 = farthest from r1; ecc(a1), b1 = farthest from a1; r2 = floor(ecc/2)
//   from a1 on the path back from b1; a2 = farthest from r2; ecc(a2), b2;
//   l = max(ecc(a1), ecc(a2)); u = floor(ecc(a2)/2) from a2 on the path back
//   from b2; i = ecc(u), lb = max(l, i), ub = 2i; then rounds while ub > lb,
//   at most three: B = the largest eccentricity over the fringe (distance i
//   from u, searched 64 sources at a time); if max(lb, B) > 2(i - 1) the
//   bound is exact, else lb = max(lb, B), ub = 2(i - 1), i = i - 1.
// Two launches: the first search of every block (small workgroups, all
// blocks resident), then the rest for the connected blocks only, listed by
// the first launch, with workgroups sized to that count (one with many
// searches must not run on a few waves).  `levels` takes the most levels
// any block's searches ran.
template <int NT>
__global__ __launch_bounds__(NT) void k_diam_first(const int64_t* row_ptr, const int32_t* col,
                                                   const int32_t* A, GraphDev g, int32_t* dist,
                                                   int32_t* qa_all, int32_t* qb_all,
                                                   int32_t* levels)
{
    __shared__ DiamShared sh;
    const int32_t b = blockIdx.x;
    const int32_t size = g.size[b];
    if (size == 0) return;   // reported as 0 from the size alone
    if (threadIdx.x == 0) sh.levels = 0;
    const int32_t off = g.moff[b];
    const InputView gv{row_ptr, col, A, g.mem, b};
    bfs_block<NT>(gv, off, size, g.seed[b], dist, qa_all + off, qb_all + off, sh);
    if (threadIdx.x == 0) {
        const bool conn = sh.reached == size;
        g.conn[b] = conn ? 1 : 0;
        g.far1[b] = g.al[far_vertex(sh.far)].y;
        g.nlev[b] = sh.levels;
        if (conn) g.clist[atomicAdd(g.ccount, 1)] = b;
        atomicMax(levels, sh.levels);
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_diam_rest(GraphDev g, int32_t* dist, int32_t* du,
                                                  int32_t* qa_all, int32_t* qb_all,
                                                  int32_t* fr_all, unsigned long long* seen,
                                                  unsigned long long* arr0,
                                                  unsigned long long* arr1, int32_t* levels)
{
    __shared__ DiamShared sh;
    const int32_t b = g.clist[blockIdx.x];
    const int tid = threadIdx.x;
    const int32_t size = g.size[b];
    if (tid == 0) sh.levels = g.nlev[b];
    const int32_t off = g.moff[b];
    int32_t* qa = qa_all + off;
    int32_t* qb = qb_all + off;
    const LocalView gv{g.lrp, g.lcol, g.mem};
    auto search = [&](int32_t src, int32_t* d) { bfs_block<NT>(gv, off, size, src, d, qa, qb, sh); };
    // the farthest vertex of the last search, as a local id
    auto far = [&]() -> int32_t { return g.al[far_vertex(sh.far)].y; };
    // the vertex `steps` closer to the search's source on the path back from x
    auto back = [&](const int32_t* d, int32_t x, int32_t steps) -> int32_t {
        if (tid == 0) sh.src = walk_back(g, d, x, steps);
        __syncthreads();
        const int32_t v = sh.src;
        __syncthreads();
        return v;
    };
    search(g.far1[b], dist);                             // from a1
    const int32_t e1 = far_level(sh.far);
    search(back(dist, far(), e1 - e1 / 2), dist);        // from r2
    search(far(), dist);                                 // from a2
    const int32_t e2 = far_level(sh.far);
    const int32_t lval = max(e1, e2);
    search(back(dist, far(), e2 - e2 / 2), du);          // from u
    int32_t i = far_level(sh.far);
    int32_t lb = max(lval, i), ub = 2 * i;
    int32_t* fr = fr_all + off;   // the fringe
    for (int round = 0; round < 3 && ub > lb; ++round) {
        if (tid == 0) sh.fcount = 0;
        __syncthreads();
        for (int j = tid; j < size; j += NT)
            if (du[off + j] == i) fr[atomicAdd(&sh.fcount, 1)] = off + j;
        __syncthreads();
        const int nf = sh.fcount;
        int32_t B = -1;
        for (int t0 = 0; t0 < nf; t0 += 64) {
            mbfs_block<NT>(g, off, size, fr + t0, min(64, nf - t0), seen, arr0, arr1, qa, qb, sh);
            B = max(B, sh.blast);
        }
        const int32_t m = max(lb, B);
        if (m > 2 * (i - 1)) {
            lb = m;
            ub = m;
        } else {
            lb = m;
            ub = 2 * (i - 1);
            i = i - 1;
        }
    }
    if (tid == 0) {
        g.ecc1[b] = e1;
        g.lval[b] = lval;
        g.fi[b] = i;
        g.lb[b] = lb;
        g.ub[b] = ub;
        atomicMax(levels, sh.levels);
    }
}

// Offsets of the blocks' vertex lists: exclusive prefix sums of the block
// sizes (one block of 1024 threads, each over a contiguous segment); the
// cursor of every list to 0.
__global__ __launch_bounds__(1024) void k_block_offsets(int k, GraphDev g)
{
    __shared__ int32_t sh[1024];
    const int per = (k + 1023) / 1024;
    const int b0 = (int)threadIdx.x * per;
    int32_t s = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < k) s += g.size[b0 + q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int32_t v = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = sh[threadIdx.x] - s;
    for (int q = 0; q < per; ++q)
        if (b0 + q < k) {
            g.moff[b0 + q] = run;
            g.fill[b0 + q] = 0;
            run += g.size[b0 + q];
        }
    if (threadIdx.x == 1023) g.moff[k] = sh[1023];
}

// Every vertex into its block's list (order within a list is free: nothing
// depends on it).
__global__ __launch_bounds__(kBlock) void k_block_members(int64_t n, const int32_t* A, GraphDev g)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const int32_t a = A[v];
    const int32_t i = g.moff[a] + atomicAdd(&g.fill[a], 1);
    g.mem[i] = (int32_t)v;
    g.al[v] = make_int2(a, i);
}

// Rows of the relabelled subgraphs of the connected blocks (the others need
// no more searches): the intra-block degree of every local id (from the
// vertex pass; 0 in a disconnected block), then, after their exclusive scan
// into lrp, each vertex's own-block neighbours as local ids, in the order of
// its input row.
__global__ __launch_bounds__(kBlock) void k_local_deg(int64_t n, GraphDev g, int32_t* dl)
{
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= n) return;
    const int2 av = g.al[v];
    dl[av.y] = g.conn[av.x] ? g.ldeg[v] : 0;
}

__global__ __launch_bounds__(kBlock) void k_local_fill(int64_t n, const int64_t* row_ptr,
                                                       const int32_t* col, GraphDev g)
{
    const int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (u >= n) return;
    const int2 au = g.al[u];
    if (!g.conn[au.x]) return;
    int64_t pos = g.lrp[au.y];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
        const int2 aw = g.al[col[e]];   // one 8-byte read: block and local id
        if (aw.x == au.x) g.lcol[pos++] = aw.y;
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
hipError_t launch_knn_d(const RunDev& r, const KnnPts& P, int K, int32_t* nbr,
                        unsigned long long* visits, hipStream_t s)
{
    const unsigned grid = nblocks(r.ngroups, kBlock / kWave);
    switch (K) {
#define BKM_KNN_CASE(KK) \
    case KK: k_knn<D, KK><<<grid, kBlock, 0, s>>>(r, P, nbr, visits); break;
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

hipError_t launch_knn(const RunDev& r, const KnnPts& P, int K, int32_t* nbr,
                      unsigned long long* visits, hipStream_t s)
{
    // a tile's parts are tested one per lane
    if (r.T / kWave * kKnnParts > kWave || !P.pbox) return hipErrorInvalidValue;
    return r.d == 2 ? launch_knn_d<2>(r, P, K, nbr, visits, s)
                    : launch_knn_d<3>(r, P, K, nbr, visits, s);
}

hipError_t launch_knn_partbox(const RunDev& r, const KnnPts& P, double* hb, hipStream_t s)
{
    const unsigned grid = nblocks(r.ngroups, kBlock / kWave);
    if (r.d == 2) k_knn_partbox<2><<<grid, kBlock, 0, s>>>(r, P, hb);
    else k_knn_partbox<3><<<grid, kBlock, 0, s>>>(r, P, hb);
    return hipGetLastError();
}

hipError_t launch_knn_widen(const RunDev& r, double* x, hipStream_t s)
{
    k_knn_widen<<<nblocks(r.npad, kBlock), kBlock, 0, s>>>(r, x);
    return hipGetLastError();
}

hipError_t launch_order_check(int64_t n, const int32_t* order, int32_t* mark, int* bad,
                              hipStream_t s)
{
    k_order_mark<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, order, mark, bad);
    k_order_check<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, mark, bad);
    return hipGetLastError();
}

hipError_t launch_sym_count(int64_t n, int K, const int32_t* nbr, const int32_t* order,
                            int32_t* extra, unsigned long long* miss, int* bad, hipStream_t s)
{
    k_sym_count<<<nblocks(n * K, kBlock), kBlock, 0, s>>>(n, K, nbr, order, extra, miss, bad);
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

hipError_t launch_sym_fill(int64_t n, int K, const int32_t* nbr, const int32_t* order,
                           const unsigned long long* miss, const int64_t* row_ptr,
                           int32_t* cursor, int32_t* col, hipStream_t s)
{
    k_sym_copy<<<nblocks(n * K, kBlock), kBlock, 0, s>>>(n, K, nbr, row_ptr, col);
    k_sym_fill<<<nblocks(n * K, kBlock), kBlock, 0, s>>>(n, K, nbr, order, miss, row_ptr, cursor,
                                                         col);
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

hipError_t launch_block_lists(int64_t n, const int32_t* A, int k, const GraphDev& g, hipStream_t s)
{
    k_block_offsets<<<1, 1024, 0, s>>>(k, g);
    k_block_members<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, A, g);
    return hipGetLastError();
}

hipError_t launch_local_rows(int64_t n, const int64_t* row_ptr, const int32_t* col,
                             const int32_t* A, const GraphDev& g, int32_t* dl, int64_t* part,
                             hipStream_t s)
{
    k_local_deg<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, g, dl);
    hipError_t e = launch_sym_rows(n, 0, dl, part, g.lrp, s);
    if (e != hipSuccess) return e;
    k_local_fill<<<nblocks(n, kBlock), kBlock, 0, s>>>(n, row_ptr, col, g);
    return hipGetLastError();
}

// Workgroup size for `blocks` workgroups: all resident at once where
// possible (2048 threads per CU), 64 to 1024 threads each.
static int diam_threads(int blocks)
{
    const int64_t per = (int64_t)256 * 2048 / std::max(blocks, 1);
    return per >= 1024 ? 1024 : per >= 512 ? 512 : per >= 256 ? 256 : per >= 128 ? 128 : 64;
}

hipError_t launch_diam_first(const int64_t* row_ptr, const int32_t* col, const int32_t* A, int k,
                             const GraphDev& g, int32_t* dist, int32_t* qa, int32_t* qb,
                             int32_t* levels, hipStream_t s)
{
    switch (diam_threads(k)) {
#define BKM_DIAM_FIRST(NT) \
    case NT: k_diam_first<NT><<<k, NT, 0, s>>>(row_ptr, col, A, g, dist, qa, qb, levels); break;
        BKM_DIAM_FIRST(1024) BKM_DIAM_FIRST(512) BKM_DIAM_FIRST(256) BKM_DIAM_FIRST(128)
        BKM_DIAM_FIRST(64)
#undef BKM_DIAM_FIRST
    }
    return hipGetLastError();
}

hipError_t launch_diam_rest(int nconn, const GraphDev& g, int32_t* dist, int32_t* du, int32_t* qa,
                            int32_t* qb, int32_t* fr, unsigned long long* seen,
                            unsigned long long* arr0, unsigned long long* arr1, int32_t* levels,
                            hipStream_t s)
{
    if (nconn <= 0) return hipSuccess;
    switch (diam_threads(nconn)) {
#define BKM_DIAM_REST(NT)                                                                   \
    case NT:                                                                                \
        k_diam_rest<NT><<<nconn, NT, 0, s>>>(g, dist, du, qa, qb, fr, seen, arr0, arr1, levels); \
        break;
        BKM_DIAM_REST(1024) BKM_DIAM_REST(512) BKM_DIAM_REST(256) BKM_DIAM_REST(128)
        BKM_DIAM_REST(64)
#undef BKM_DIAM_REST
    }
    return hipGetLastError();
}

hipError_t launch_gm_final(int k, const GraphDev& g, int32_t* diam_out, int32_t* diam_ub_out,
                           int64_t* comm_out, double* summary, hipStream_t s)
{
    k_gm_final<<<1, 1024, 0, s>>>(k, g, diam_out, diam_ub_out, comm_out, summary);
    return hipGetLastError();
}

}  // namespace bkm
