// Assignment sweep of balanced k-means (Alg. 1 inner loop; Sec. 4.2-4.4).
//
// Every point takes the center with the smallest effective distance
// dist(p, c) / influence(c).  Two exact prunings from the paper, laid out for
// the GPU:
//   * centers (Sec. 4.4): for a box B of points, a center whose smallest
//     possible effective distance to B exceeds the second-smallest largest
//     effective distance of any center to B can be neither the best nor the
//     second-best center of any point in B.  The filter runs at two levels:
//     super-tiles against all k centers (k_supercand, one block each), then
//     every tile of consecutive Hilbert-ordered points against its
//     super-tile's list (k_tilecand, one wave each), which writes the
//     surviving centers as compact records: FP32 offset from the tile anchor
//     and squared FP32 inverse influence.
//   * points (Sec. 4.3, Hamerly): a point whose upper bound on the effective
//     distance to its own center is below its lower bound on the second-best
//     effective distance keeps its block without evaluating anything.  The
//     bounds are stored lazily -- the upper bound as a distance relative to the
//     accumulated movement of its center, the lower bound in a global affine
//     frame (M, E) -- so a point that is skipped is never written.
// The sweep itself (k_sweep) streams the points' block ids and bounds; points
// the bounds settle stop there, the others are compacted into a per-tile work
// list in LDS and each gets a full lane to scan the tile's records (staged in
// LDS).  Block weights are maintained incrementally: a point that changes
// block moves its exact fixed-point weight (a count for unit weights) from
// the old to the new block with integer atomics, so the weights equal the
// from-scratch sums bit for bit whatever the scheduling order.
#include <math.h>

#include "bkm_internal.h"

namespace bkm {

namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24, unit roundoff of FP32
constexpr double kFixPt2 = 1.53e-05;               // >= 1.0001 * 2^-16: 16-bit point offsets, times Rn
constexpr double kFixPt3 = 4.77e-07;               // >= 1.0001 * 2^-21: 21-bit point offsets, times Rn
constexpr double kCandSlack = 1e-9;               // relative slack of the center filter
constexpr double kTiny = 1e-12;                   // relative slack of FP64 bound arithmetic
constexpr double kInf = INFINITY;
// Absolute slack of the FP32 screen: squared distances or effective squared
// distances below 2^-126 may lose relative accuracy (subnormal range), which
// moves their square roots by less than 2^-62.
constexpr double kUnder = 0x1p-60;
// The screen takes square roots with the hardware instruction (v_sqrt_f32):
// within 1 ulp (2u relative) for arguments of at least 2^-96, and within
// kSqrtAbs absolutely below that (the root of such an argument is < 2^-48).
// The FP32 value v of a candidate's effective squared distance has a
// correctly rounded root within [e(1-8u) - tau, e(1+8u) + tau] of the exact
// effective distance e; so its raw root r satisfies
//   r(1 - kScr) - slack <= e <= r(1 + kScr) + slack,
//   slack = tau(1 + 16u) + 2 kSqrtAbs,
// and a raw root of any value below v gives a lower bound the same way.
constexpr double kSqrtAbs = 0x1p-47;
constexpr double kScr = 11.0 * kU32;

__device__ inline float sqrt_raw(float x) { return __builtin_amdgcn_sqrtf(x); }

// Squared smallest and largest effective distance from center c to the box
// [lo, hi]; iv = 1 / influence(c).
template <int D>
__device__ inline void box_eff2(const double* lo, const double* hi, const double* C, int k,
                                int c, double iv, double& lo2, double& hi2)
{
    double mn = 0.0, mx = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double cj = C[(int64_t)j * k + c];
        const double g = fmax(fmax(lo[j] - cj, cj - hi[j]), 0.0);
        const double f = fmax(fabs(cj - lo[j]), fabs(cj - hi[j]));
        mn += g * g;
        mx += f * f;
    }
    const double iv2 = iv * iv;
    lo2 = mn * iv2;
    hi2 = mx * iv2;
}

// Effective distance in FP64, evaluated exactly as defined:
// sqrt((dx*dx + dy*dy) + dz*dz) / influence, no fused multiply-add (the
// library is compiled with -ffp-contract=off).
template <int D>
__device__ inline double eff64(const double* x, double cx, double cy, double cz, double infl,
                               double& sq)
{
    const double dx = x[0] - cx;
    const double dy = x[1] - cy;
    double s = dx * dx + dy * dy;
    if (D == 3) {
        const double dz = x[2] - cz;
        s = s + dz * dz;
    }
    sq = s;
    return sqrt(s) / infl;
}

__device__ inline double sorted_coord(const RunDev& r, int j, int64_t p)
{
    return r.in_f32 ? (double)r.xs32[j][p] : r.xs64[j][p];
}

// ------------------------------------------------- hyper- and super-tiles
// Candidate filter of one box [lo, hi] against the centers of `list` (all k
// centers when list is NULL): c stays iff its smallest effective distance to
// the box is at most the second-smallest largest one (Sec. 4.4: no point of
// the box can have c as best or second-best otherwise).  A box inside a
// parent box may filter the parent's list instead of all centers: its
// smallest distances are no smaller and its second-smallest largest distance
// is no larger, so every center the parent drops it drops too, and the two
// centers of its smallest largest distances are on the parent's list.
template <int D, int NT, typename RT>
__device__ __forceinline__ void box_filter(RT r, const double* lo, const double* hi,
                                           const int* __restrict__ list, int L, int* out,
                                           int* count_out)
{
    __shared__ double sa[NT / kWave], sb[NT / kWave];
    __shared__ int cnt;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int k = r.k;
    Two t{kInf, kInf};
    for (int i = tid; i < L; i += NT) {
        const int c = list ? list[i] : i;
        double lo2, hi2;
        box_eff2<D>(lo, hi, r.C, k, c, r.clus[c].y, lo2, hi2);
        t = merge_two(t, Two{hi2, kInf});
    }
    t = wave_two(t);
    if (lane == 0) {
        sa[wv] = t.a;
        sb[wv] = t.b;
    }
    if (tid == 0) cnt = 0;
    __syncthreads();
    Two all{sa[0], sb[0]};
    for (int w = 1; w < NT / kWave; ++w) all = merge_two(all, Two{sa[w], sb[w]});
    const double thr2 = all.b * (1.0 + 2.0 * kCandSlack);
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int i0 = 0; i0 < L; i0 += NT) {
        const int i = i0 + tid;
        int c = 0;
        bool keep = false;
        if (i < L) {
            c = list ? list[i] : i;
            double lo2, hi2;
            box_eff2<D>(lo, hi, r.C, k, c, r.clus[c].y, lo2, hi2);
            keep = lo2 <= thr2;
        }
        const unsigned long long b = __ballot(keep);
        int off = 0;
        if (lane == 0 && b) off = atomicAdd(&cnt, (int)__popcll(b));
        off = __shfl(off, 0, kWave);
        if (keep) out[off + __popcll(b & below)] = c;
    }
    __syncthreads();
    if (tid == 0) *count_out = cnt;
}

// Hyper-tiles (kHyper super-tiles) against all k centers: few blocks with
// long lists, so each block has kHyperThreads threads.
constexpr int kHyperThreads = 1024;

template <int D, typename RT>
__device__ __forceinline__ void hypercand_body(RT r, const int bid)
{
    const DevState* st = r.st;
    if (st->done || st->round_done) return;
    double lo[D], hi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lo[j] = r.hbox[(int64_t)bid * 2 * D + j];
        hi[j] = r.hbox[(int64_t)bid * 2 * D + D + j];
    }
    box_filter<D, kHyperThreads, RT>(r, lo, hi, nullptr, r.k, r.hlist + (int64_t)bid * r.k, r.hcount + bid);
}

template <int D>
__global__ __launch_bounds__(kHyperThreads) void k_hypercand(RunDev r)
{
    hypercand_body<D, const RunDev>(r, blockIdx.x);
}

template <int D>
__global__ __launch_bounds__(kHyperThreads) void k_hypercand_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    hypercand_body<D, const RunDev&>(rs[m.x], m.y);
}

// Super-tiles against their hyper-tile's list, kSuperThreads threads each.
constexpr int kSuperThreads = 512;

template <int D, typename RT>
__device__ __forceinline__ void supercand_body(RT r, const int bid)
{
    const DevState* st = r.st;
    if (st->done || st->round_done) return;
    double lo[D], hi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lo[j] = r.sbox[(int64_t)bid * 2 * D + j];
        hi[j] = r.sbox[(int64_t)bid * 2 * D + D + j];
    }
    const int h = bid / kHyper;
    box_filter<D, kSuperThreads, RT>(r, lo, hi, r.hlist + (int64_t)h * r.k, r.hcount[h],
                      r.slist + (int64_t)bid * r.k, r.scount + bid);
}

template <int D>
__global__ __launch_bounds__(kSuperThreads) void k_supercand(RunDev r)
{
    supercand_body<D, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
template <int D>
__global__ __launch_bounds__(kSuperThreads) void k_supercand_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    supercand_body<D, const RunDev&>(rs[m.x], m.y);
}

// ------------------------------------------------------------------ tiles
// One wave per tile: filter the super-tile list against the tile box and
// write the survivors' records plus the FP32 error bounds of the tile.
//
// FP32 error bound.  Points enter the FP32 screen as fixed-point offsets
// from the tile anchor X (tile box center): on axis j in units of h_j/M, h_j
// the box half-extent, rounded to nearest, with M = 2^15 - 1 (2D, 16-bit
// fields) or 2^20 - 1 (3D, 21-bit fields), so each stored coordinate is
// within h_j/(2M) of exact and the point within 1.0001*Rn/(2M), Rn the norm of
// the half-extents (2^-16 resp. 2^-21 relative).  The FP32 value of a point
// coordinate (unit times integer, the unit itself rounded) adds 2*u*Rn
// (u = 2^-24); the FP32 center offset is within 1.0001*u*r_c, r_c the
// distance of center c from X; the FP32 difference and norm (two fused
// multiply-adds and a square root) add at most 3.6*u*(Rn + r_c).  dmax uses
// Rn/(2M)*1.0001 + 8*u*(Rn + r_c), and tau that times 1/influence(c),
// maximised over the candidates.
template <int D, int PREC, typename RT>
__device__ __forceinline__ void tilecand_body(RT r, const int bid)
{
    const DevState* st = r.st;
    if (st->done || st->round_done) return;
    constexpr int kCpl = 4;   // candidates a lane keeps in registers between passes
    const int lane = threadIdx.x % kWave;
    // wave-uniform: the tile box, its frame and the list bounds live in scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(bid * (kBlock / kWave) + (int)threadIdx.x / kWave);
    if (tile >= r.ntiles) return;
    const int k = r.k;
    const double* __restrict__ C = r.C;

    double blo[D], bhi[D], X[D];
    double rn2 = 0.0;
    float step[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < D; ++j) {
        blo[j] = r.tbox[(int64_t)tile * 2 * D + j];
        bhi[j] = r.tbox[(int64_t)tile * 2 * D + D + j];
        X[j] = 0.5 * (blo[j] + bhi[j]);
        const double h = fmax(bhi[j] - X[j], X[j] - blo[j]);
        rn2 += h * h;
        step[j] = (float)(h / FixPack<D>::kMax);
    }
    const double Rn = sqrt(rn2) * (1.0 + kTiny);
    const double pnt = (D == 3 ? kFixPt3 : kFixPt2) * Rn;   // fixed-point term of the bound
    const int sidx = tile / r.super_tiles;
    const int L = r.scount[sidx];
    const int* __restrict__ sl = r.slist + (int64_t)sidx * k;
    CandRec* __restrict__ out = r.tcand + (int64_t)tile * kTileCap;
    const unsigned long long below = (1ULL << lane) - 1ULL;

    int cnt = 0;
    double tau = 0.0, dmax = 0.0;
    // error bounds of one candidate; the record itself when it fits
    auto emit = [&](bool keep, int c) {
        const unsigned long long b = __ballot(keep);
        const int pos = cnt + (int)__popcll(b & below);
        if (keep) {
            const double iv = r.clus[c].y;
            double dd = 0.0, q[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                q[j] = C[(int64_t)j * k + c] - X[j];
                dd += q[j] * q[j];
            }
            const double delta = pnt + 8.0 * kU32 * (Rn + sqrt(dd) * (1.0 + kTiny)) + kUnder;
            dmax = fmax(dmax, delta);
            tau = fmax(tau, delta * iv);
            if (pos < kTileCap) {
                CandRec rec;
                rec.qx = (float)q[0];
                rec.qy = (float)q[1];
                rec.qz = D == 3 ? (float)q[D - 1] : 0.0f;
                const float fi = (float)iv;
                rec.w2 = fi * fi;
                rec.id = c;
                rec.pad0 = rec.pad1 = rec.pad2 = 0;
                out[pos] = rec;
            }
        }
        cnt += (int)__popcll(b);
    };

    Two t{kInf, kInf};
    double thr2;
    if (L <= kCpl * kWave) {
        int cc[kCpl];
        double clo[kCpl];
#pragma unroll
        for (int u = 0; u < kCpl; ++u) {
            const int i = lane + u * kWave;
            cc[u] = -1;
            clo[u] = kInf;
            if (i < L) {
                const int c = sl[i];
                double lo2, hi2;
                box_eff2<D>(blo, bhi, C, k, c, r.clus[c].y, lo2, hi2);
                cc[u] = c;
                clo[u] = lo2;
                t = merge_two(t, Two{hi2, kInf});
            }
        }
        t = wave_two(t);
        thr2 = t.b * (1.0 + 2.0 * kCandSlack);
#pragma unroll
        for (int u = 0; u < kCpl; ++u) emit(cc[u] >= 0 && clo[u] <= thr2, cc[u]);
    } else {
        for (int i = lane; i < L; i += kWave) {
            const int c = sl[i];
            double lo2, hi2;
            box_eff2<D>(blo, bhi, C, k, c, r.clus[c].y, lo2, hi2);
            t = merge_two(t, Two{hi2, kInf});
        }
        t = wave_two(t);
        thr2 = t.b * (1.0 + 2.0 * kCandSlack);
        for (int i0 = 0; i0 < L; i0 += kWave) {
            const int i = i0 + lane;
            int c = 0;
            bool keep = false;
            if (i < L) {
                c = sl[i];
                double lo2, hi2;
                box_eff2<D>(blo, bhi, C, k, c, r.clus[c].y, lo2, hi2);
                keep = lo2 <= thr2;
            }
            emit(keep, c);
        }
    }
    // an overflowed tile is swept in FP64 over the super-tile list (its
    // FP32 bounds are not used)
    const bool overflow = cnt > kTileCap;
    tau = wave_max_d(tau);
    dmax = wave_max_d(dmax);
    if (lane == 0) {
        TileHead h;
        h.n = overflow ? 0 : cnt;
        h.overflow = overflow ? 1 : 0;
        h.tau = tau * (1.0 + kTiny) + kUnder;
        h.dmax = dmax * (1.0 + kTiny);
        h.lb_out = sqrt(t.b) * (1.0 - kTiny);
        h.step[0] = step[0];
        h.step[1] = step[1];
        h.step[2] = step[2];
        h.pad = 0.0f;
        r.thead[tile] = h;
    }
}

template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void k_tilecand(RunDev r)
{
    tilecand_body<D, PREC, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
template <int D, int PREC>
__global__ __launch_bounds__(kBlock) void k_tilecand_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    tilecand_body<D, PREC, const RunDev&>(rs[m.x], m.y);
}

// ------------------------------------------------------------------ sweep
// Block = one tile of T = 256 * PPT consecutive Hilbert-ordered points.
// Phase 1 streams every point of the tile (thread t, points base + t + 256 q,
// so each wave reads 64 consecutive points and every access is coalesced):
// block id, stored bounds, Hamerly test.  The points the bounds cannot
// decide are compacted into an LDS work list, and phase 2 gives each of them
// a full lane for the candidate scan (records staged in LDS), the decision
// and the block-weight bookkeeping, so skipped points cost no candidate
// arithmetic.  The coordinate sums of the center update are not touched
// here: the round-end pass rebuilds them from the final assignment.
template <int D, int PREC, int PPT, bool WEIGHTED, typename RT>
__device__ __forceinline__ void sweep_body(RT r, const int bid)
{
    DevState* st = r.st;
    if (st->done || st->round_done) return;
    constexpr bool F32 = PREC == BKM_PREC_F32_RECHECK;
    constexpr int T = kBlock * PPT;
    __shared__ int s_off[T];      // tile offsets of the points to evaluate
    __shared__ int s_aold[T];     // and their current block
    __shared__ int s_gflag[T / kWave];  // per 64-point group: common block, or -1
    __shared__ int s_gdirty[T / kWave]; // per 64-point group: a point of it changed block
    __shared__ float4 s_q[kTileCap];
    __shared__ int s_cid[kTileCap];
    __shared__ double s_c64[4][kTileCap];   // FP64 centers and influences (FP64 sweep, overflow)
    __shared__ int s_nl;
    __shared__ unsigned long long s_cnt[kBlock / kWave][5];   // counters of each wave

    const int tid = threadIdx.x, lane = tid % kWave;
    const int tile = bid;
    const int64_t base = (int64_t)tile * T;
    const int k = r.k;
    const double* __restrict__ C = r.C;
    const double* __restrict__ I = r.I;
    if (tid == 0) s_nl = 0;
    if (tid < T / kWave) s_gdirty[tid] = 0;

    // ---- phase 1: block ids and stored bounds (arrays are padded to whole tiles)
    int aold[PPT];
    float ut[PPT], lt[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * kBlock + tid;
        aold[q] = r.A[p];
        ut[q] = r.use_bounds ? r.ubt[p] : 0.0f;
        lt[q] = r.use_bounds ? r.lbt[p] : 0.0f;
    }
    const TileHead hd = r.thead[tile];
    const int sidx = tile / r.super_tiles;
    const int* __restrict__ sl = r.slist + (int64_t)sidx * k;
    const CandRec* __restrict__ cr = r.tcand + (int64_t)tile * kTileCap;
    const int ncand = hd.overflow ? r.scount[sidx] : hd.n;
    // the tile's candidate records into LDS
    if (!hd.overflow && tid < hd.n) {
        const CandRec rec = cr[tid];
        s_cid[tid] = rec.id;
        if (F32) {
            s_q[tid] = make_float4(rec.qx, rec.qy, rec.qz, rec.w2);
        } else {
            s_c64[0][tid] = C[rec.id];
            s_c64[1][tid] = C[(int64_t)k + rec.id];
            s_c64[2][tid] = D == 3 ? C[(int64_t)(D - 1) * k + rec.id] : 0.0;
            s_c64[3][tid] = I[rec.id];
        }
    }
    float2 cl[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) cl[q] = r.clus32[aold[q] > 0 ? aold[q] : 0];
    // lower-bound frame in FP32, rounded so that every bound stays valid, and
    // the reciprocal of its scale (precomputed by whoever changed the frame)
    const float Mf = st->Mf, Ef = st->Ef;
    const double E = st->E;
    const double invM = st->invM;
    unsigned n_eval = 0, n_skip = 0;
    __syncthreads();   // s_nl initialised
    const unsigned long long below = (1ULL << lane) - 1ULL;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        bool ev = aold[q] != kPad && ncand > 0;
        bool sk = false;
        if (ev && r.use_bounds && aold[q] >= 0) {
            // Hamerly test (Sec. 4.3): upper bound on the own effective
            // distance below the lower bound on the second-best one.  FP32
            // with absolute slack covering every rounding.
            float sub = ut[q] + cl[q].x;
            sub += 0x1p-21f * (fabsf(ut[q]) + cl[q].x);
            const float ub = sub * cl[q].y * (1.0f + 0x1p-20f);
            const float m = Mf * lt[q];
            const float lb = (m - Ef) - 0x1p-20f * (m + Ef);
            if (ub < lb) {
                ev = false;
                sk = true;
            }
        }
        const unsigned long long b = __ballot(ev);
        // counters are wave-uniform: popcounts of ballots
        n_skip += (unsigned)__popcll(__ballot(sk));
        n_eval += (unsigned)__popcll(b);
        int pos = 0;
        if (lane == 0 && b) pos = atomicAdd(&s_nl, (int)__popcll(b));
        pos = __shfl(pos, 0, kWave) + (int)__popcll(b & below);
        if (ev) {
            s_off[pos] = q * kBlock + tid;
            s_aold[pos] = aold[q];
        }
        // the wave holds one whole 64-point group here: its common block
        const int a0 = __shfl(aold[q], 0, kWave);
        const bool same = __ballot(aold[q] != a0) == 0ULL;
        if (lane == 0) s_gflag[q * (kBlock / kWave) + tid / kWave] = same ? a0 : -1;
    }
    __syncthreads();
    const int nl = s_nl;

    // ---- phase 2: one lane per undecided point
    unsigned n_rechk = 0, n_chg = 0;
    const double gap_rel = r.recheck_gap;
    const double wsc = st->w_scale;
    // an overflowed tile (more candidates than records) is swept in FP64
    // even by the FP32 kernel: its candidates come from the super-tile list,
    // and without a tile-sized error bound the screen would send most
    // points to the recheck
    const bool screen = F32 && !hd.overflow;
    for (int i0 = 0; i0 < nl; i0 += kBlock) {
        const int i = i0 + tid;
        const bool act = i < nl;
        const int off = act ? s_off[i] : 0;
        const int ao = act ? s_aold[i] : -1;
        const int64_t p = base + off;
        float o[D];
        double x[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            o[j] = 0.0f;
            x[j] = 0.0;
        }
        if (act) {
            if (screen) {
                // one load per point: its packed fixed-point offsets
                const auto w = static_cast<const typename FixPack<D>::word*>(r.ofs)[p];
#pragma unroll
                for (int j = 0; j < D; ++j) o[j] = fix_field<D>(w, j) * hd.step[j];
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) x[j] = sorted_coord(r, j, p);
            }
        }
        // best and second-best over the tile's candidates
        float b2 = INFINITY, s2 = INFINITY;
        int bi = 0;
        double be = kInf, se = kInf, bs2 = kInf;
        int bc = 0x7fffffff;
        // FP32 squared distance (scaled units) and effective squared distance
        auto eff32 = [&](float qx, float qy, float qz, float w2, float& d2) {
            const float dx = o[0] - qx;
            const float dy = o[1] - qy;
            d2 = dx * dx;
            d2 = __builtin_fmaf(dy, dy, d2);
            if (D == 3) {
                const float dz = o[D - 1] - qz;
                d2 = __builtin_fmaf(dz, dz, d2);
            }
            return d2 * w2;
        };
        // the FP32 record of candidate c0 of the tile
        auto rec32 = [&](int c0, int& c, float& qx, float& qy, float& qz, float& w2) {
            c = s_cid[c0];
            const float4 qv = s_q[c0];
            qx = qv.x;
            qy = qv.y;
            qz = qv.z;
            w2 = qv.w;
        };
        // best and second-best FP32 values with b2 <= s2: the new second is
        // the median of (b2, s2, e2); only the best's record index is kept
        auto consider32 = [&](int c0, float qx, float qy, float qz, float w2) {
            float d2;
            const float e2 = eff32(qx, qy, qz, w2, d2);
            const bool better = e2 < b2;
            s2 = __builtin_amdgcn_fmed3f(b2, s2, e2);
            bi = better ? c0 : bi;
            b2 = better ? e2 : b2;
        };
        // the same ranking by squared effective distance, iv2 = (1/influence)^2
        auto consider64sq = [&](int c, double cx, double cy, double cz, double iv2) {
            const double dx = x[0] - cx;
            const double dy = x[1] - cy;
            double sq = dx * dx + dy * dy;
            if (D == 3) {
                const double dz = x[2] - cz;
                sq = sq + dz * dz;
            }
            const double e2 = sq * iv2;
            const bool better = e2 < be || (e2 == be && c < bc);
            se = better ? be : fmin(se, e2);
            bs2 = better ? sq : bs2;
            bc = better ? c : bc;
            be = better ? e2 : be;
        };
        auto consider64 = [&](int c, double cx, double cy, double cz, double ic) {
            double sq;
            const double e = eff64<D>(x, cx, cy, cz, ic, sq);
            const bool better = e < be || (e == be && c < bc);
            se = better ? be : fmin(se, e);
            bs2 = better ? sq : bs2;
            bc = better ? c : bc;
            be = better ? e : be;
        };
        if (!hd.overflow) {
            if (__ballot(act) != 0ULL) {
                for (int c0 = 0; c0 < ncand; ++c0) {
                    const int c = s_cid[c0];
                    if (F32) {
                        const float4 qv = s_q[c0];
                        consider32(c0, qv.x, qv.y, qv.z, qv.w);
                    } else {
                        consider64(c, s_c64[0][c0], s_c64[1][c0], s_c64[2][c0], s_c64[3][c0]);
                    }
                }
            }
        } else {
            // overflowed tile: the super-tile's list in FP64, staged through
            // LDS in chunks of kTileCap centers that every wave of the block
            // helps to load (the loop is block-uniform).  Candidates are
            // compared by their squared effective distance s * (1/I)^2, with
            // no square root or division per candidate: its rounding differs
            // from sqrt(s) / I by a few units of 2^-53, which can only swap
            // two candidates closer than that (a tie at the 1e-12 level), and
            // the bounds below carry a 1e-12 slack.
            for (int cb = 0; cb < ncand; cb += kTileCap) {
                const int m = min(kTileCap, ncand - cb);
                __syncthreads();   // the previous chunk is consumed
                if (tid < m) {
                    const int c = sl[cb + tid];
                    const double iv = r.clus[c].y;
                    s_cid[tid] = c;
                    s_c64[0][tid] = C[c];
                    s_c64[1][tid] = C[(int64_t)k + c];
                    s_c64[2][tid] = D == 3 ? C[(int64_t)(D - 1) * k + c] : 0.0;
                    s_c64[3][tid] = iv * iv;
                }
                __syncthreads();
                if (__ballot(act) != 0ULL) {
                    for (int c0 = 0; c0 < m; ++c0)
                        consider64sq(s_cid[c0], s_c64[0][c0], s_c64[1][c0], s_c64[2][c0], s_c64[3][c0]);
                }
            }
            // back to effective distances for the lower bound
            se = sqrt(se);
        }
        int cbest = ao;
        bool chg = false, rck = false;
        long long wh = 1, wl = 0;
        if (act) {
            double ubd, lb;
            if (screen) {
                // the best candidate's id, FP32 effective squared distance and
                // squared distance, recomputed from its record exactly as in
                // the loop
                float bd2, be2;
                {
                    float qx, qy, qz, w2;
                    rec32(bi, bc, qx, qy, qz, w2);
                    be2 = eff32(qx, qy, qz, w2, bd2);
                }
                // every other candidate's FP32 value is at least s2
                const double eb = (double)sqrt_raw(be2);
                const double es = (double)sqrt_raw(s2);
                const double slack = hd.tau * (1.0 + 16.0 * kU32) + 2.0 * kSqrtAbs;
                // one candidate: certain; an overflowed FP32 value: decide in FP64
                const bool sure =
                    b2 < INFINITY &&
                    (ncand == 1 ||
                     (s2 < INFINITY &&
                      es * (1.0 - kScr) - eb * (1.0 + kScr) > 2.0 * slack &&
                      es - eb > gap_rel * es));
                if (sure) {
                    cbest = bc;
                    ubd = ((double)sqrt_raw(bd2) + 2.0 * kSqrtAbs) * (1.0 + 7.0 * kU32) + hd.dmax;
                    lb = es * (1.0 - kScr) - slack;
                } else {
                    // FP64 recheck of the candidates that can still be the best:
                    // every candidate's exact effective distance e lies within
                    // [r(1-kScr) - slack, r(1+kScr) + slack] of its raw FP32
                    // root r, so the exact best has r(1-kScr) <= eb(1+kScr) +
                    // 2 slack (the window), and every candidate outside it is
                    // farther than window - slack.
                    rck = true;
#pragma unroll
                    for (int j = 0; j < D; ++j) x[j] = sorted_coord(r, j, p);
                    const double win = eb * (1.0 + kScr) + 2.0 * slack;
                    double b = kInf, s = kInf, bsq = kInf;
                    int bcc = 0x7fffffff;
                    for (int c0 = 0; c0 < ncand; ++c0) {
                        int c;
                        float qx, qy, qz, w2, d2;
                        rec32(c0, c, qx, qy, qz, w2);
                        const float e32 = sqrt_raw(eff32(qx, qy, qz, w2, d2));
                        if (!((double)e32 * (1.0 - kScr) <= win)) continue;
                        double sq;
                        const double e = eff64<D>(x, C[c], C[(int64_t)k + c],
                                                  D == 3 ? C[(int64_t)(D - 1) * k + c] : 0.0, I[c], sq);
                        if (e < b || (e == b && c < bcc)) {
                            s = b;
                            b = e;
                            bcc = c;
                            bsq = sq;
                        } else if (e < s) {
                            s = e;
                        }
                    }
                    cbest = bcc;
                    ubd = sqrt(bsq) * (1.0 + kTiny);
                    lb = fmin(s, win - slack) * (1.0 - kTiny);
                }
            } else {
                cbest = bc;
                ubd = sqrt(bs2) * (1.0 + kTiny);
                lb = se * (1.0 - kTiny);
            }
            if (cbest < 0 || cbest >= k) cbest = ao >= 0 ? ao : (hd.overflow ? sl[0] : s_cid[0]);
            lb = fmin(lb, hd.lb_out);
            if (r.use_bounds) {
                const double Db = r.clus[cbest].x;
                double uv = ubd - Db;
                uv += kTiny * (fabs(ubd) + Db);
                r.ubt[p] = f32_up(uv);
                double lv = (lb + E) * invM;
                lv -= kTiny * fabs(lv);
                r.lbt[p] = (lv > 0.0) ? f32_down(lv) : 0.0f;
            }
            if (cbest != ao) {
                chg = true;
                r.A[p] = cbest;
                s_gflag[off / kWave] = -1;   // conservatively mixed from now on
                s_gdirty[off / kWave] = 1;
                if (WEIGHTED) fix_split(r.ws[p] * wsc, wh, wl);
            }
        }
        n_rechk += (unsigned)__popcll(__ballot(rck));
        // wave-aggregated transfer of the point's weight from the old to the new block
        unsigned long long pend = __ballot(chg);
        n_chg += (unsigned)__popcll(pend);
        while (pend) {
            const int leader = __builtin_ctzll(pend);
            const int ka = __shfl(ao, leader, kWave);
            const int kb = __shfl(cbest, leader, kWave);
            const bool mine = chg && ao == ka && cbest == kb;
            const unsigned long long mm = __ballot(mine);
            long long vh, vl = 0;
            if (WEIGHTED) {
                vh = wave_sum_ll(mine ? wh : 0);
                vl = wave_sum_ll(mine ? wl : 0);
            } else {
                vh = (long long)__popcll(mm);
            }
            if (lane == leader) {
                unsigned long long* nb = (unsigned long long*)(r.acc + (int64_t)kb * kAcc + kAccW);
                atomicAdd(nb, (unsigned long long)vh);
                if (WEIGHTED) atomicAdd(nb + 1, (unsigned long long)vl);
                if (ka >= 0) {
                    unsigned long long* ob = (unsigned long long*)(r.acc + (int64_t)ka * kAcc + kAccW);
                    atomicAdd(ob, (unsigned long long)(-vh));
                    if (WEIGHTED) atomicAdd(ob + 1, (unsigned long long)(-vl));
                }
            }
            pend &= ~mm;
        }
    }

    // counters: per wave in LDS, then per block one slot of 64 (never a single address)
    if (lane == 0) {
        const int wv = tid / kWave;
        s_cnt[wv][0] = n_eval;
        s_cnt[wv][1] = n_skip;
        s_cnt[wv][2] = n_rechk;
        s_cnt[wv][3] = n_chg;
        s_cnt[wv][4] = (unsigned long long)n_eval * (unsigned long long)ncand;
    }
    __syncthreads();
    // per 64-point group: the common block of its points (or -1, also when a
    // point of it changed block in this sweep), for the round-end pass
    if (tid < T / kWave) {
        r.gblk[base / kWave + tid] = s_gflag[tid];
        // the round-end pass moves the coordinate sums of these groups' points
        if (s_gdirty[tid]) r.gdirty[base / kWave + tid] = 1;
    }
    if (tid < 5) {
        unsigned long long v = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) v += s_cnt[w][tid];
        unsigned long long* slot = r.cnt + (int64_t)(tile % kCntSlots) * kCntWords;
        if (v) atomicAdd(slot + tid, v);
    }
    if (tid == 0 && hd.overflow) {
        unsigned long long* slot = r.cnt + (int64_t)(tile % kCntSlots) * kCntWords;
        atomicAdd(slot + kCntOverflow, 1ULL);
    }
}

template <int D, int PREC, int PPT, bool WEIGHTED>
__global__ __launch_bounds__(kBlock, 7) void k_sweep(RunDev r)
{
    sweep_body<D, PREC, PPT, WEIGHTED, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
template <int D, int PREC, int PPT, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_sweep_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    sweep_body<D, PREC, PPT, WEIGHTED, const RunDev&>(rs[m.x], m.y);
}

template <int D, int PREC, bool WEIGHTED>
hipError_t sweep_ppt(const RunDev& r, hipStream_t s)
{
    switch (r.ppt) {
    case 1: k_sweep<D, PREC, 1, WEIGHTED><<<r.ntiles, kBlock, 0, s>>>(r); break;
    case 2: k_sweep<D, PREC, 2, WEIGHTED><<<r.ntiles, kBlock, 0, s>>>(r); break;
    default: k_sweep<D, PREC, 4, WEIGHTED><<<r.ntiles, kBlock, 0, s>>>(r); break;
    }
    return hipGetLastError();
}

template <int D, int PREC>
hipError_t sweep_w(const RunDev& r, hipStream_t s)
{
    return r.weighted ? sweep_ppt<D, PREC, true>(r, s) : sweep_ppt<D, PREC, false>(r, s);
}

template <int D>
hipError_t sweep_p(const RunDev& r, hipStream_t s)
{
    return r.precision == BKM_PREC_F32_RECHECK ? sweep_w<D, BKM_PREC_F32_RECHECK>(r, s)
                                               : sweep_w<D, BKM_PREC_F64>(r, s);
}

}  // namespace

hipError_t launch_supercand(const RunDev& r, hipStream_t s)
{
    if (r.d == 2) {
        k_hypercand<2><<<r.nhyper, kHyperThreads, 0, s>>>(r);
        k_supercand<2><<<r.nsuper, kSuperThreads, 0, s>>>(r);
    } else {
        k_hypercand<3><<<r.nhyper, kHyperThreads, 0, s>>>(r);
        k_supercand<3><<<r.nsuper, kSuperThreads, 0, s>>>(r);
    }
    return hipGetLastError();
}

hipError_t launch_tilecand(const RunDev& r, hipStream_t s)
{
    const unsigned g = (unsigned)((r.ntiles + kBlock / kWave - 1) / (kBlock / kWave));
    const bool f32 = r.precision == BKM_PREC_F32_RECHECK;
    if (r.d == 2) {
        if (f32) k_tilecand<2, BKM_PREC_F32_RECHECK><<<g, kBlock, 0, s>>>(r);
        else k_tilecand<2, BKM_PREC_F64><<<g, kBlock, 0, s>>>(r);
    } else {
        if (f32) k_tilecand<3, BKM_PREC_F32_RECHECK><<<g, kBlock, 0, s>>>(r);
        else k_tilecand<3, BKM_PREC_F64><<<g, kBlock, 0, s>>>(r);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const RunDev& r, hipStream_t s)
{
    return r.d == 2 ? sweep_p<2>(r, s) : sweep_p<3>(r, s);
}

template <int D, int PREC, bool WEIGHTED>
hipError_t sweep_multi_ppt(const MultiSet& m, hipStream_t s)
{
    switch (m.ppt) {
    case 1: k_sweep_multi<D, PREC, 1, WEIGHTED><<<m.nb_tile, kBlock, 0, s>>>(m.rs, m.map_tile); break;
    case 2: k_sweep_multi<D, PREC, 2, WEIGHTED><<<m.nb_tile, kBlock, 0, s>>>(m.rs, m.map_tile); break;
    default: k_sweep_multi<D, PREC, 4, WEIGHTED><<<m.nb_tile, kBlock, 0, s>>>(m.rs, m.map_tile); break;
    }
    return hipGetLastError();
}

template <int D, int PREC>
hipError_t sweep_multi_p(const MultiSet& m, hipStream_t s)
{
    if (m.nb_hyper) k_hypercand_multi<D><<<m.nb_hyper, kHyperThreads, 0, s>>>(m.rs, m.map_hyper);
    if (m.nb_super) k_supercand_multi<D><<<m.nb_super, kSuperThreads, 0, s>>>(m.rs, m.map_super);
    if (m.nb_quad) k_tilecand_multi<D, PREC><<<m.nb_quad, kBlock, 0, s>>>(m.rs, m.map_quad);
    if (!m.nb_tile) return hipGetLastError();
    return m.weighted ? sweep_multi_ppt<D, PREC, true>(m, s) : sweep_multi_ppt<D, PREC, false>(m, s);
}

hipError_t launch_sweep_multi(const MultiSet& m, hipStream_t s)
{
    const bool f32 = m.precision == BKM_PREC_F32_RECHECK;
    if (m.d == 2)
        return f32 ? sweep_multi_p<2, BKM_PREC_F32_RECHECK>(m, s) : sweep_multi_p<2, BKM_PREC_F64>(m, s);
    return f32 ? sweep_multi_p<3, BKM_PREC_F32_RECHECK>(m, s) : sweep_multi_p<3, BKM_PREC_F64>(m, s);
}

}  // namespace bkm
