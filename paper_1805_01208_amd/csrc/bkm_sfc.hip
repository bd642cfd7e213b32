// Hilbert space-filling-curve bootstrap of balanced k-means (Alg. 2: the SFC
// index of every point, the stable sort by it, the redistribution into
// sorted order and the initial centers; Sec. 4.1).  On one GPU the global sort
// and redistribution become an LSD radix sort of (key, index) followed by one
// gather into a structure-of-arrays copy in curve order, cut into tiles of
// consecutive points whose bounding boxes drive the candidate pruning of the
// sweep.
#include <math.h>

#include "bkm_internal.h"

namespace bkm {

namespace {

template <typename T>
__device__ inline double ld(const void* p, int64_t i)
{
    return (double)((const T*)p)[i];
}

// ---------------------------------------------------------------- bbox
// Per-block partial min/max of every axis, the largest weight and finiteness
// checks; a single block then folds the partials into the run state.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bbox_partial(RunDev r)
{
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    double wmax = 0.0, wsum = 0.0;
    int bad = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < r.n; i += stride) {
        for (int j = 0; j < r.d; ++j) {
            double v = ld<T>(r.in_x[j], i);
            if (!isfinite(v)) bad = 1;
            mn[j] = fmin(mn[j], v);
            mx[j] = fmax(mx[j], v);
        }
        if (r.in_w) {
            double w = r.in_w[i];
            if (!(w > 0.0) || !isfinite(w)) bad = 1;
            wmax = fmax(wmax, w);
            wsum += w;
        }
    }
    __shared__ double sh[kBlock / kWave][8];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int j = 0; j < 3; ++j) {
        mn[j] = wave_min_d(mn[j]);
        mx[j] = wave_max_d(mx[j]);
    }
    wmax = wave_max_d(wmax);
    wsum = wave_sum_d(wsum);
    unsigned long long anybad = __ballot(bad);
    if (lane == 0) {
        for (int j = 0; j < 3; ++j) {
            sh[wv][j] = mn[j];
            sh[wv][3 + j] = mx[j];
        }
        sh[wv][6] = wmax;
        sh[wv][7] = wsum;
        if (anybad) atomicOr(&r.st->bad_data, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double o[8];
        for (int q = 0; q < 8; ++q) o[q] = sh[0][q];
        for (int w = 1; w < kBlock / kWave; ++w) {
            for (int j = 0; j < 3; ++j) {
                o[j] = fmin(o[j], sh[w][j]);
                o[3 + j] = fmax(o[3 + j], sh[w][3 + j]);
            }
            o[6] = fmax(o[6], sh[w][6]);
            o[7] += sh[w][7];
        }
        for (int q = 0; q < 8; ++q) r.red[(int64_t)blockIdx.x * 8 + q] = o[q];
    }
}

// The partials folded by all threads (thread t over parts t, t + 256, ...,
// then a fixed tree over the threads: the weight sum's order is fixed).
__global__ __launch_bounds__(kBlock) void k_bbox_final(RunDev r, int nparts, int m)
{
    __shared__ double sh[kBlock][8];
    double f[8] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        const double* p = r.red + (int64_t)b * 8;
        for (int j = 0; j < 3; ++j) {
            f[j] = fmin(f[j], p[j]);
            f[3 + j] = fmax(f[3 + j], p[3 + j]);
        }
        f[6] = fmax(f[6], p[6]);
        f[7] += p[7];
    }
    for (int q = 0; q < 8; ++q) sh[threadIdx.x][q] = f[q];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double* a = sh[threadIdx.x];
            const double* b = sh[threadIdx.x + w];
            for (int j = 0; j < 3; ++j) {
                a[j] = fmin(a[j], b[j]);
                a[3 + j] = fmax(a[3 + j], b[3 + j]);
            }
            a[6] = fmax(a[6], b[6]);
            a[7] += b[7];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double* o = sh[0];
        DevState* st = r.st;
        double ext = 0.0;
        for (int j = 0; j < 3; ++j) {
            st->lo[j] = j < r.d ? o[j] : 0.0;
            st->hi[j] = j < r.d ? o[3 + j] : 0.0;
            if (j < r.d && o[3 + j] - o[j] > ext) ext = o[3 + j] - o[j];
        }
        st->ext = ext;
        st->key_scale = ext > 0.0 ? ldexp(1.0, m) / ext : 0.0;
        // fixed-point scales: every coordinate term w*(x-lo)*sx_scale and
        // weight term w*w_scale stays below 2^61 (power-of-two scales, so
        // scaling is exact and only the final rounding to an integer is not)
        double wmax = r.in_w ? o[6] : 1.0;
        double span = ext > 0.0 ? ext * wmax : wmax;
        st->sx_scale = ldexp(1.0, 60 - ilogb(span));
        st->w_scale = r.in_w ? ldexp(1.0, 60 - ilogb(wmax)) : 1.0;
        st->wmax = wmax;
        st->total_weight = r.in_w ? o[7] : (double)r.n;
    }
}

// ---------------------------------------------------------------- Hilbert
// Hilbert index of cell (q0..q_{d-1}) at order m (Skilling, "Programming the
// Hilbert curve", 2004): axes -> transposed index by walking levels from the
// top (set bit in axis i: invert the lower bits of axis 0; clear bit:
// exchange the lower bits of axes 0 and i), Gray code across axes, then
// remove the accumulated rotation; finally interleave the transposed bits,
// top level first, axis 0 first.
template <int D>
__device__ inline uint64_t hilbert_key(uint32_t* q, int m)
{
    for (int lvl = m - 1; lvl >= 1; --lvl) {
        const uint32_t hb = 1u << lvl;
        const uint32_t below = hb - 1u;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (q[a] & hb) {
                q[0] ^= below;
            } else {
                const uint32_t sw = (q[0] ^ q[a]) & below;
                q[0] ^= sw;
                q[a] ^= sw;
            }
        }
    }
#pragma unroll
    for (int a = 1; a < D; ++a) q[a] ^= q[a - 1];
    uint32_t rot = 0;
    for (int lvl = m - 1; lvl >= 1; --lvl)
        if (q[D - 1] & (1u << lvl)) rot ^= (1u << lvl) - 1u;
#pragma unroll
    for (int a = 0; a < D; ++a) q[a] ^= rot;
    uint64_t key = 0;
    for (int lvl = m - 1; lvl >= 0; --lvl) {
#pragma unroll
        for (int a = 0; a < D; ++a) key = (key << 1) | (uint64_t)((q[a] >> lvl) & 1u);
    }
    return key;
}

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_keys(RunDev r, int m, uint64_t* keys,
                                                 int32_t* vals)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= r.n) return;
    const DevState* st = r.st;
    uint64_t key = 0;
    if (st->ext > 0.0) {
        const double scale = st->key_scale;
        const double top = ldexp(1.0, m) - 1.0;
        uint32_t q[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double c = floor((ld<T>(r.in_x[a], i) - st->lo[a]) * scale);
            q[a] = (uint32_t)fmin(c, top);
        }
        key = hilbert_key<D>(q, m);
    }
    keys[i] = key;
    vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------- radix sort
// Stable LSD radix sort of (64-bit key, int32 value), 8-bit digits.  Per pass:
// block histograms (digit-major), one exclusive scan, then a stable scatter in
// which every block ranks its items in input order with wave ballots.
constexpr int kIpt = kSortIpt;
constexpr int kChunk = kSortChunk;
constexpr int kScanSeg = 1024;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t* keys, int64_t n,
                                                      int shift, uint32_t* hist, int nblk)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int it = 0; it < kIpt; ++it) {
        int64_t i = base + (int64_t)it * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `len` counts, three kernels: segment sums, a scan of the
// segment sums in one block, then the scan inside each segment.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t* in, int64_t len,
                                                       uint32_t* part)
{
    __shared__ uint32_t sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanSeg;
    uint32_t s = 0;
    for (int q = threadIdx.x; q < kScanSeg; q += kBlock)
        if (base + q < len) s += in[base + q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(1024) void k_scan_top(uint32_t* part, int nseg)
{
    __shared__ uint32_t sh[1024];
    const int per = (nseg + 1023) / 1024;
    const int b = threadIdx.x * per;
    uint32_t s = 0;
    for (int q = 0; q < per; ++q)
        if (b + q < nseg) s += part[b + q];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = sh[threadIdx.x] - s;  // exclusive
    for (int q = 0; q < per; ++q)
        if (b + q < nseg) {
            uint32_t v = part[b + q];
            part[b + q] = run;
            run += v;
        }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t* data, int64_t len,
                                                     const uint32_t* part)
{
    __shared__ uint32_t sh[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanSeg;
    constexpr int per = kScanSeg / kBlock;
    uint32_t v[per];
    uint32_t s = 0;
    for (int q = 0; q < per; ++q) {
        int64_t i = base + (int64_t)threadIdx.x * per + q;
        v[q] = i < len ? data[i] : 0;
        s += v[q];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        uint32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = part[blockIdx.x] + sh[threadIdx.x] - s;
    for (int q = 0; q < per; ++q) {
        int64_t i = base + (int64_t)threadIdx.x * per + q;
        if (i < len) data[i] = run;
        run += v[q];
    }
}

// Stable scatter of one block's chunk: the items are first placed in LDS in
// (digit, input order) order, then written out so that each digit's items
// leave as one contiguous run (coalesced stores).  offs is the scanned
// histogram (digit-major): this block's items of digit d go to offs[d][blk]
// onwards, and offs[d][blk+1] - offs[d][blk] of them exist.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t* kin,
                                                         const int32_t* vin, uint64_t* kout,
                                                         int32_t* vout, int64_t n, int shift,
                                                         const uint32_t* offs, int nblk)
{
    __shared__ uint64_t lk[kChunk];
    __shared__ int32_t lv[kChunk];
    __shared__ uint32_t lstart[256];   // chunk-local start of each digit
    __shared__ uint32_t lrun[256];     // next chunk-local slot of each digit
    __shared__ uint32_t goff[256];     // global position of the block's first item per digit
    __shared__ uint32_t wc[kBlock / kWave][256];
    __shared__ uint32_t wsum[kBlock / kWave];
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    const int64_t idx = (int64_t)t * nblk + blockIdx.x;
    const int64_t len = (int64_t)256 * nblk;
    const uint32_t g0 = offs[idx];
    const uint32_t cnt = (idx + 1 < len ? offs[idx + 1] : (uint32_t)n) - g0;
    goff[t] = g0;
    // exclusive scan of the block's digit counts (256 = kBlock threads)
    uint32_t x = cnt;
    for (int m = 1; m < kWave; m <<= 1) {
        const uint32_t y = __shfl_up(x, m, kWave);
        if (lane >= m) x += y;
    }
    if (lane == kWave - 1) wsum[wv] = x;
    for (int w = 0; w < kBlock / kWave; ++w) wc[w][t] = 0;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wv; ++w) pre += wsum[w];
    lstart[t] = pre + x - cnt;
    lrun[t] = pre + x - cnt;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int it = 0; it < kIpt; ++it) {
        const int64_t i = base + (int64_t)it * kBlock + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0;
        const int32_t val = valid ? vin[i] : 0;
        const uint32_t dig = (uint32_t)((key >> shift) & 255u);
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bal = __ballot((dig >> b) & 1u);
            same &= ((dig >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (valid && rank == 0) wc[wv][dig] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t lp = lrun[dig] + rank;
            for (int w = 0; w < wv; ++w) lp += wc[w][dig];
            lk[lp] = key;
            lv[lp] = val;
        }
        __syncthreads();
        uint32_t tot = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            tot += wc[w][t];
            wc[w][t] = 0;
        }
        lrun[t] += tot;
        __syncthreads();
    }
    const int64_t m = n - base < kChunk ? n - base : kChunk;
    for (int j = t; j < m; j += kBlock) {
        const uint64_t key = lk[j];
        const uint32_t d = (uint32_t)((key >> shift) & 255u);
        const uint32_t gp = goff[d] + ((uint32_t)j - lstart[d]);
        kout[gp] = key;
        vout[gp] = lv[j];
    }
}

// ---------------------------------------------------------------- permute
// Coordinates in Hilbert order (no padding yet).
template <typename T>
// One axis per grid row (blockIdx.y), so each gather works on one
// coordinate array at a time.
__global__ __launch_bounds__(kBlock) void k_permute(RunDev r)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= r.n) return;
    const int32_t s = r.sperm[i];
    const int j = blockIdx.y;
    if (r.in_f32)
        r.tx32[j][i] = ((const float*)r.in_x[j])[s];
    else
        r.tx64[j][i] = ((const double*)r.in_x[j])[s];
}

__device__ inline double tx_at(const RunDev& r, int j, int64_t i)
{
    return r.in_f32 ? (double)r.tx32[j][i] : r.tx64[j][i];
}

// ---------------------------------------------------------------- jumps
// The Hilbert order keeps consecutive points close, except where the curve
// leaves the data and re-enters elsewhere (empty parts of the curve's cube).
// A tile straddling such a jump gets a huge box and a huge candidate list, so
// the layout is padded to start a new tile after every jump.  A jump is a gap
// between consecutive points larger than 64 times the median gap (median from
// a histogram of binary exponents of the squared gaps, so the threshold is
// exact and order-independent; the comparisons take squared gaps).
__device__ inline int gap_bin(double g2)
{
    if (!(g2 > 0.0)) return 0;
    const int e = (ilogb(g2) >> 1) + 64;   // the exponent of the gap, rounded down
    return e < 1 ? 1 : (e >= kGapBins ? kGapBins - 1 : e);
}

__device__ inline double gap2_at(const RunDev& r, int64_t i)
{
    double s = 0.0;
    for (int j = 0; j < r.d; ++j) {
        const double v = tx_at(r, j, i + 1) - tx_at(r, j, i);
        s += v * v;
    }
    return s;
}

__global__ __launch_bounds__(kBlock) void k_gap_hist(RunDev r)
{
    __shared__ unsigned int h[kGapBins];
    if (threadIdx.x < kGapBins) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i + 1 < r.n; i += stride)
        atomicAdd(&h[gap_bin(gap2_at(r, i))], 1u);
    __syncthreads();
    if (threadIdx.x < kGapBins && h[threadIdx.x]) atomicAdd(&r.ghist[threadIdx.x], h[threadIdx.x]);
}

// The jump threshold, squared, into the run state: the upper edge of the
// median bin times 64 (0: no jumps).
__global__ __launch_bounds__(kWave) void k_gap_threshold(RunDev r)
{
    if (threadIdx.x != 0) return;
    unsigned long long tot = 0, acc = 0;
    for (int b = 0; b < kGapBins; ++b) tot += r.ghist[b];
    int med = 0;
    for (int b = 0; b < kGapBins; ++b) {
        acc += r.ghist[b];
        if (2 * acc >= tot) { med = b; break; }
    }
    const double thr = med == 0 ? 0.0 : ldexp(1.0, med - 64 + 1 + 6);
    r.st->jump_thr2 = thr * thr;
}

__global__ __launch_bounds__(kBlock) void k_jump_find(RunDev r)
{
    const double thr2 = r.st->jump_thr2;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i + 1 >= r.n || !(thr2 > 0.0)) return;
    if (gap2_at(r, i) > thr2) {
        const int slot = atomicAdd(&r.st->njumps, 1);
        if (slot < r.maxjumps) r.jumps[slot] = (int32_t)(i + 1);
    }
}

// One block: sort the jump starts, then walk them to give every run its
// layout shift (the padding that moves its first point to a tile boundary).
__global__ __launch_bounds__(1024) void k_jump_plan(RunDev r)
{
    __shared__ int32_t sj[kMaxJumps];
    DevState* st = r.st;
    const int nj = min(st->njumps, r.maxjumps);
    int m = 1;
    while (m < nj) m <<= 1;
    for (int i = threadIdx.x; i < m; i += 1024) sj[i] = i < nj ? r.jumps[i] : 0x7fffffff;
    __syncthreads();
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < m; i += 1024) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const int32_t a = sj[i], b = sj[j];
                    if ((a > b) == up) {
                        sj[i] = b;
                        sj[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        int64_t shift = 0;
        for (int q = 0; q < nj; ++q) {
            const int64_t pos = (int64_t)sj[q] + shift;
            shift += (r.T - pos % r.T) % r.T;
            r.jumps[q] = sj[q];
            r.jshift[q] = shift;
        }
        const int64_t used = r.n + shift;
        st->npad = (used + r.T - 1) / r.T * r.T;
        st->njumps = nj;
    }
}

// Index of the first jump start after Hilbert position i (binary search).
__device__ inline int jump_after(const RunDev& r, int nj, int64_t i)
{
    int lo = 0, hi = nj;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)r.jumps[mid] <= i) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_init_layout(RunDev r)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= r.npad) return;
    r.perm[p] = -1;
    r.A[p] = kPad;
}

// Points into the padded layout; the last point before each gap in the
// layout also fills the gap with copies of itself, so tile and group boxes
// are those of the real points.
// The layout shift of Hilbert position i is that of the last jump at or
// before it: one binary search per block for its first point, then a short
// forward scan per thread (a block's 256 points hold few jump starts).
__global__ __launch_bounds__(kBlock) void k_place(RunDev r)
{
    __shared__ int s_j0;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = i0 + threadIdx.x;
    const int nj = r.st->njumps;
    if (threadIdx.x == 0) s_j0 = jump_after(r, nj, i0);
    __syncthreads();
    if (i >= r.n) return;
    int j = s_j0;
    while (j < nj && (int64_t)r.jumps[j] <= i) ++j;
    const int64_t pos = i + (j > 0 ? r.jshift[j - 1] : 0);
    const int32_t src = r.sperm[i];
    r.perm[pos] = src;
    r.A[pos] = -1;
    if (r.ws) r.ws[pos] = r.in_w[src];
    double x[3];
    for (int j = 0; j < r.d; ++j) {
        x[j] = tx_at(r, j, i);
        if (r.in_f32)
            r.xs32[j][pos] = r.tx32[j][i];
        else
            r.xs64[j][pos] = x[j];
    }
    int jn = j;
    while (jn < nj && (int64_t)r.jumps[jn] <= i + 1) ++jn;
    const int64_t next = (i + 1 < r.n) ? i + 1 + (jn > 0 ? r.jshift[jn - 1] : 0) : r.npad;
    for (int64_t q = pos + 1; q < next; ++q) {
        for (int j = 0; j < r.d; ++j) {
            if (r.in_f32)
                r.xs32[j][q] = r.tx32[j][i];
            else
                r.xs64[j][q] = x[j];
        }
    }
}

__device__ inline double xs_at(const RunDev& r, int j, int64_t i)
{
    return r.in_f32 ? (double)r.xs32[j][i] : r.xs64[j][i];
}

// Per tile (one block of T sorted points): exact FP64 box, boxes of its
// 64-point groups, and the fixed-point offsets of its points from the box
// center.
template <int D>
__global__ __launch_bounds__(kBlock) void k_tile_prep(RunDev r)
{
    __shared__ double sh[kBlock / kWave][2 * D];
    __shared__ double box[2 * D];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * r.T;
    double tmn[D], tmx[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        tmn[j] = INFINITY;
        tmx[j] = -INFINITY;
    }
    for (int q = 0; q < r.ppt; ++q) {
        const int64_t g0 = base + (int64_t)q * kBlock + wv * kWave;  // group start
        const int64_t i = g0 + lane;
        double gmn[D], gmx[D];
        // the group's box: maxima of -x and x over the wave, in one pass
        double v[2 * D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double x = xs_at(r, j, i);
            v[j] = -x;
            v[D + j] = x;
        }
        wave_max_dpp<2 * D>(v);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            gmn[j] = -v[j];
            gmx[j] = v[D + j];
            tmn[j] = fmin(tmn[j], gmn[j]);
            tmx[j] = fmax(tmx[j], gmx[j]);
        }
        if (lane == 0) {
            double* gb = r.gbox + (g0 / kWave) * 2 * D;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                gb[j] = gmn[j];
                gb[D + j] = gmx[j];
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sh[wv][j] = tmn[j];
            sh[wv][D + j] = tmx[j];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * D) {
        const int j = threadIdx.x;
        double v = sh[0][j];
        for (int w = 1; w < kBlock / kWave; ++w) v = j < D ? fmin(v, sh[w][j]) : fmax(v, sh[w][j]);
        box[j] = v;
        r.tbox[(int64_t)blockIdx.x * 2 * D + j] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the frame of the packed offsets below and of the candidate filter
        TileFrame f;
        double rn2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            f.X[j] = 0.0;
            f.step[j] = 0.0f;
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double X = 0.5 * (box[j] + box[D + j]);
            const double h = fmax(box[D + j] - X, X - box[j]);
            rn2 += h * h;
            f.X[j] = X;
            f.step[j] = (float)(h / FixPack<D>::kMax);
        }
        f.hnorm = sqrt(rn2);
        f.pad = 0.0f;
        r.tframe[blockIdx.x] = f;
    }
    if (r.precision == BKM_PREC_F32_RECHECK) {
        double X[D], h[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            X[j] = 0.5 * (box[j] + box[D + j]);
            h[j] = fmax(box[D + j] - X[j], X[j] - box[j]);
        }
        for (int q = 0; q < r.ppt; ++q) {
            const int64_t i = base + (int64_t)q * kBlock + threadIdx.x;
            long long f[D];
#pragma unroll
            for (int j = 0; j < D; ++j) f[j] = fix_offset<D>(xs_at(r, j, i) - X[j], h[j]);
            static_cast<typename FixPack<D>::word*>(r.ofs)[i] = fix_pack<D>(f);
        }
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_super_boxes(RunDev r)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s >= r.nsuper) return;
    const int t0 = s * r.super_tiles;
    const int t1 = min(r.ntiles, t0 + r.super_tiles);
    double b[2 * D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        b[j] = INFINITY;
        b[D + j] = -INFINITY;
    }
    for (int t = t0; t < t1; ++t) {
        const double* tb = r.tbox + (int64_t)t * 2 * D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            b[j] = fmin(b[j], tb[j]);
            b[D + j] = fmax(b[D + j], tb[D + j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) r.sbox[(int64_t)s * 2 * D + j] = b[j];
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_hyper_boxes(RunDev r)
{
    const int h = blockIdx.x * kBlock + threadIdx.x;
    if (h >= r.nhyper) return;
    const int s0 = h * kHyper;
    const int s1 = min(r.nsuper, s0 + kHyper);
    double b[2 * D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        b[j] = INFINITY;
        b[D + j] = -INFINITY;
    }
    for (int s = s0; s < s1; ++s) {
        const double* sb = r.sbox + (int64_t)s * 2 * D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            b[j] = fmin(b[j], sb[j]);
            b[D + j] = fmax(b[D + j], sb[D + j]);
        }
    }
#pragma unroll
    for (int j = 0; j < 2 * D; ++j) r.hbox[(int64_t)h * 2 * D + j] = b[j];
}

// Initial centers (Alg. 2): center c is the sorted point
// floor(c*n/k) + floor(n/(2k)); with target sizes t it is
// floor(n*S_c/tsum) + floor(n*t_c/(2 tsum)), at most n-1, S_c the prefix sum.
__global__ __launch_bounds__(kBlock) void k_centers_from_sorted(RunDev r, double* out,
                                                               int row_major)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= r.k) return;
    int64_t pos;
    if (r.tsz) {
        // the middle of the c-th stretch when the curve is cut in
        // proportion to the target sizes
        const double tsum = r.tpre[r.k];
        pos = (int64_t)floor(((double)r.n * r.tpre[c]) / tsum) +
              (int64_t)floor(((double)r.n * r.tsz[c]) / (2.0 * tsum));
        if (pos > r.n - 1) pos = r.n - 1;
    } else {
        pos = ((int64_t)c * r.n) / r.k + r.n / (2 * (int64_t)r.k);
    }
    for (int j = 0; j < r.d; ++j) {
        double v = tx_at(r, j, pos);
        if (row_major)
            out[(int64_t)c * r.d + j] = v;
        else
            out[(int64_t)j * r.k + c] = v;
    }
}

inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_bbox(const RunDev& r, int hilbert_order, hipStream_t s)
{
    int nparts = (int)std::min<int64_t>(4096, (r.n + kBlock - 1) / kBlock);
    if (r.in_f32)
        k_bbox_partial<float><<<nparts, kBlock, 0, s>>>(r);
    else
        k_bbox_partial<double><<<nparts, kBlock, 0, s>>>(r);
    k_bbox_final<<<1, kBlock, 0, s>>>(r, nparts, hilbert_order);
    return hipGetLastError();
}

hipError_t launch_keys(const RunDev& r, int hilbert_order, int32_t* vals, hipStream_t s)
{
    unsigned g = nblocks(r.n, kBlock);
    if (r.d == 2) {
        if (r.in_f32) k_keys<float, 2><<<g, kBlock, 0, s>>>(r, hilbert_order, r.keys, vals);
        else k_keys<double, 2><<<g, kBlock, 0, s>>>(r, hilbert_order, r.keys, vals);
    } else {
        if (r.in_f32) k_keys<float, 3><<<g, kBlock, 0, s>>>(r, hilbert_order, r.keys, vals);
        else k_keys<double, 3><<<g, kBlock, 0, s>>>(r, hilbert_order, r.keys, vals);
    }
    return hipGetLastError();
}

// Sorts (keys, vals) on their low `nbits` bits; the result ends in keys/vals.
hipError_t radix_sort_pairs(const RunDev& r, uint64_t* keys, int32_t* vals, int nbits,
                            hipStream_t s)
{
    const int64_t n = r.n;
    const int nblk = (int)nblocks(n, kChunk);
    const int64_t len = (int64_t)256 * nblk;
    const int nseg = (int)((len + kScanSeg - 1) / kScanSeg);
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = r.keys2;
    int32_t* vb = r.vals2;
    int passes = (nbits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        k_radix_hist<<<nblk, kBlock, 0, s>>>(ka, n, shift, r.hist, nblk);
        k_scan_reduce<<<nseg, kBlock, 0, s>>>(r.hist, len, r.part);
        k_scan_top<<<1, 1024, 0, s>>>(r.part, nseg);
        k_scan_down<<<nseg, kBlock, 0, s>>>(r.hist, len, r.part);
        k_radix_scatter<<<nblk, kBlock, 0, s>>>(ka, va, kb, vb, n, shift, r.hist, nblk);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        hipError_t e = hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_permute(const RunDev& r, hipStream_t s)
{
    const dim3 g(nblocks(r.n, kBlock), (unsigned)r.d);
    k_permute<double><<<g, kBlock, 0, s>>>(r);
    return hipGetLastError();
}

// Gap histogram, jump search and plan; the padded size lands in st->npad.
hipError_t launch_jump_plan(const RunDev& r, hipStream_t s)
{
    hipError_t e = hipMemsetAsync(r.ghist, 0, kGapBins * sizeof(unsigned int), s);
    if (e != hipSuccess) return e;
    const unsigned g = (unsigned)std::min<int64_t>(2048, nblocks(r.n, kBlock));
    k_gap_hist<<<g, kBlock, 0, s>>>(r);
    k_gap_threshold<<<1, kWave, 0, s>>>(r);
    k_jump_find<<<nblocks(r.n, kBlock), kBlock, 0, s>>>(r);
    k_jump_plan<<<1, 1024, 0, s>>>(r);
    return hipGetLastError();
}

hipError_t launch_place(const RunDev& r, hipStream_t s)
{
    k_init_layout<<<nblocks(r.npad, kBlock), kBlock, 0, s>>>(r);
    k_place<<<nblocks(r.n, kBlock), kBlock, 0, s>>>(r);
    return hipGetLastError();
}

hipError_t launch_tile_prep(const RunDev& r, hipStream_t s)
{
    if (r.d == 2) {
        k_tile_prep<2><<<r.ntiles, kBlock, 0, s>>>(r);
        k_super_boxes<2><<<nblocks(r.nsuper, kBlock), kBlock, 0, s>>>(r);
        k_hyper_boxes<2><<<nblocks(r.nhyper, kBlock), kBlock, 0, s>>>(r);
    } else {
        k_tile_prep<3><<<r.ntiles, kBlock, 0, s>>>(r);
        k_super_boxes<3><<<nblocks(r.nsuper, kBlock), kBlock, 0, s>>>(r);
        k_hyper_boxes<3><<<nblocks(r.nhyper, kBlock), kBlock, 0, s>>>(r);
    }
    return hipGetLastError();
}

hipError_t launch_centers_from_sorted(const RunDev& r, double* out, int row_major,
                                      hipStream_t s)
{
    k_centers_from_sorted<<<nblocks(r.k, kBlock), kBlock, 0, s>>>(r, out, row_major);
    return hipGetLastError();
}

// ------------------------------------------------- random-sample order
// Key of point i for the random order: output i of splitmix64 seeded with
// `seed` (Steele, Lea, Flood, "Fast splittable pseudorandom number
// generators", 2014): state seed + (i+1)*golden gamma, then the 64-bit mixer.
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_sample_keys(RunDev r, uint64_t seed,
                                                         const uint64_t* given)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= r.n) return;
    r.keys[i] = given ? given[i] : splitmix64_at(seed, (uint64_t)i);
    r.sperm[i] = (int32_t)i;
}

hipError_t launch_sample_order(const RunDev& r, uint64_t seed, const uint64_t* given,
                               hipStream_t s)
{
    k_sample_keys<<<nblocks(r.n, kBlock), kBlock, 0, s>>>(r, seed, given);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return radix_sort_pairs(r, r.keys, r.sperm, 64, s);
}

// ---------------------------------------------- samples in Hilbert order
// A sample round only needs its points in some spatially coherent order (its
// results do not depend on the order), so the nested samples are taken from
// the full run's Hilbert layout instead of being sorted again: the layout
// positions whose point ranks below s in the random order, kept in layout
// order.

// rank[order[j]] = j: every point's position in the random order
__global__ __launch_bounds__(kBlock) void k_sample_rank(const int32_t* order, int64_t n,
                                                       int32_t* rank)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j < n) rank[order[j]] = (int32_t)j;
}

// rank of the point at each layout position; INT32_MAX for padding
__global__ __launch_bounds__(kBlock) void k_sample_layout_rank(RunDev r, const int32_t* rank,
                                                              int32_t* rk)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= r.npad) return;
    const int32_t src = r.perm[p];
    rk[p] = src >= 0 ? rank[src] : INT32_MAX;
}

// per chunk of kChunk layout positions (each thread kSortIpt consecutive
// ones): how many rank below s
__global__ __launch_bounds__(kBlock) void k_sample_count(const int32_t* rk, int64_t npad,
                                                        int64_t s, uint32_t* cnt)
{
    __shared__ uint32_t sh[kBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kSortIpt;
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSortIpt; ++q) {
        const int64_t p = base + q;
        c += (p < npad && rk[p] < s) ? 1u : 0u;
    }
    for (int m = kWave / 2; m > 0; m >>= 1) c += __shfl_xor(c, m, kWave);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += sh[w];
        cnt[blockIdx.x] = t;
    }
}

// stable compaction: the kept positions of each chunk, in layout order, from
// the chunk's scanned offset on; their coordinates and weights gathered
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sample_scatter(RunDev r, const int32_t* rk, int64_t s,
                                                          const uint32_t* off, T* x0, T* x1,
                                                          T* x2, double* w)
{
    __shared__ uint32_t sh[kBlock];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)tid * kSortIpt;
    bool keep[kSortIpt];
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSortIpt; ++q) {
        const int64_t p = base + q;
        keep[q] = p < r.npad && rk[p] < s;
        c += keep[q] ? 1u : 0u;
    }
    // exclusive scan of the threads' counts
    sh[tid] = c;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const uint32_t v = tid >= o ? sh[tid - o] : 0u;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    int64_t t = (int64_t)off[blockIdx.x] + sh[tid] - c;
    T* const xo[3] = {x0, x1, x2};
#pragma unroll
    for (int q = 0; q < kSortIpt; ++q) {
        if (!keep[q]) continue;
        const int64_t p = base + q;
        // T is the layout's own type (float for FP32 input), so no conversion
        for (int j = 0; j < r.d; ++j) xo[j][t] = r.in_f32 ? (T)r.xs32[j][p] : (T)r.xs64[j][p];
        if (w) w[t] = r.ws[p];
        ++t;
    }
}

// identity permutation: the points are taken in their given order
__global__ __launch_bounds__(kBlock) void k_iota(int32_t* v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

hipError_t launch_sample_layout_rank(const RunDev& r, int32_t* rank, int32_t* rk, hipStream_t s)
{
    k_sample_rank<<<nblocks(r.n, kBlock), kBlock, 0, s>>>(r.sperm, r.n, rank);
    k_sample_layout_rank<<<nblocks(r.npad, kBlock), kBlock, 0, s>>>(r, rank, rk);
    return hipGetLastError();
}

hipError_t launch_sample_compact(const RunDev& r, const int32_t* rk, int64_t count, void* const* x,
                                 double* w, hipStream_t s)
{
    const int nch = (int)nblocks(r.npad, kChunk);
    const int nseg = (nch + kScanSeg - 1) / kScanSeg;
    k_sample_count<<<nch, kBlock, 0, s>>>(rk, r.npad, count, r.hist);
    k_scan_reduce<<<nseg, kBlock, 0, s>>>(r.hist, nch, r.part);
    k_scan_top<<<1, 1024, 0, s>>>(r.part, nseg);
    k_scan_down<<<nseg, kBlock, 0, s>>>(r.hist, nch, r.part);
    if (r.in_f32)
        k_sample_scatter<float><<<nch, kBlock, 0, s>>>(r, rk, count, r.hist, (float*)x[0],
                                                       (float*)x[1], (float*)x[2], w);
    else
        k_sample_scatter<double><<<nch, kBlock, 0, s>>>(r, rk, count, r.hist, (double*)x[0],
                                                        (double*)x[1], (double*)x[2], w);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* v, int64_t n, hipStream_t s)
{
    k_iota<<<nblocks(n, kBlock), kBlock, 0, s>>>(v, n);
    return hipGetLastError();
}

}  // namespace bkm
