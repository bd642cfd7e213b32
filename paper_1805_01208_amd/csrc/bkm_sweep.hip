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
//     The filters keep a margin, so the lists of a round's first sweep stay
//     complete through its balance sweeps while the influences move little
//     (the balance step checks the bound); such sweeps only refresh each
//     tile's records and error bounds for the new influences.
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
// the box can have c as best or second-best otherwise), widened by the list
// margin so that the list outlives small influence changes.  A box inside a
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
    const double thr2 = all.b * (1.0 + 2.0 * kCandSlack) * kListMargin2;
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
        const unsigned long long b = wave_ballot(keep);
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
    if (round_over(st) || st->lists_ok) return;
    // the influences the lists are built for, for the balance step's test
    for (int c = bid * kHyperThreads + (int)threadIdx.x; c < r.k; c += r.nhyper * kHyperThreads)
        r.ivb[c] = r.clus[c].y;
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
    if (round_over(st) || st->lists_ok) return;
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
//
// Sort key.  For a point of the tile, the correctly rounded root of the
// screen's value for c is at least e(1 - 8u) - tau_c (tau_c: c's own term of
// tau), e its exact effective distance, and e is at least lo_c, the smallest
// effective distance from the tile box to c; so the value itself is at least
// key_c = (lo_c(1 - 10u) - tau_c)^2 (1 - 4u) (0 when negative), rounded down.
// The FP64 sweep's value s*(1/I)^2 of a point inside the box exceeds it too.
// Records are written in ascending key order, so a sweep may stop at the
// first record whose key is at least every lane's current second-best value
// (Alg. 1 breaks the same way once the box distance passes the second-best):
// no later record can change a lane's best or second-best.
// FP32 screen slack of a tile from its tau: tau(1 + 16u) + 2^-46, rounded up.
__device__ inline float screen_slack32(double tau)
{
    return f32_up((tau * (1.0 + 16.0 * kU32) + 2.0 * kSqrtAbs) * (1.0 + 0x1p-20));
}

// A sweep that keeps the lists of the last build (every 1/influence within
// [G, F] times its value then, F <= G sqrt(kListMargin2)) brings the tile's
// records and bounds to the current influences: each record's FP32 squared
// inverse influence, recomputed as the build computes it; its key, a lower
// bound on the screen's value for its center at any point of the tile, which
// scales with the center's 1/influence (its distance and error terms both
// do), so key0 G^2 is one and the order stays; tau, retaken from the
// records' error terms; and the bound on every center left out at the
// build, lb_build G.
// The smallest ratio and largest shift (r_c, s_c) over the super-tile list
// of an overflowed tile (its candidates), per lane; m starts at 1 (a larger
// ratio only tightens, so 1 is always valid).
template <typename RT>
__device__ inline void decay_over_super(RT r, int tile, int lane, double& m, double& e)
{
    const int sidx = tile / r.super_tiles;
    const int L = r.scount[sidx];
    const int* __restrict__ sl = r.slist + (int64_t)sidx * r.k;
    for (int i = lane; i < L; i += kWave) {
        const double2 d = r.cdec[sl[i]];
        m = fmin(m, d.x);
        e = fmax(e, d.y);
    }
}

// The tile's lower-bound frame f (as loaded) relaxed by (m, e) for this
// sweep (wave-uniform values).
template <typename RT>
__device__ inline void relax_tile_bound(RT r, int tile, int lane, TileBound f, double m, double e,
                                        double lb_out)
{
    if (lane == 0) {
        tile_bound_step(f, m, e, lb_out);
        r.tbnd[tile] = f;
    }
}

template <typename RT>
__device__ inline void refresh_tile(RT r, int tile, int lane)
{
    TileHead* __restrict__ hp = r.thead + tile;
    const TileBound f0 = r.tbnd[tile];
    const int n = hp->n;   // 0 for an overflowed tile
    const double G = r.st->listG;
    const double G2 = G * G * (1.0 - 0x1p-50);
    CandRec* __restrict__ cr = r.tcand + (int64_t)tile * kTileCap;
    double tau = 0.0, m = 1.0, e = 0.0;
    for (int i = lane; i < n; i += kWave) {
        CandRec rec = cr[i];
        const double iv = r.clus[rec.id].y;
        const double2 d = r.cdec[rec.id];
        m = fmin(m, d.x);
        e = fmax(e, d.y);
        rec.w2 = screen_w2(iv);
        rec.key = f32_down((double)rec.key0 * G2);
        tau = fmax(tau, (double)rec.dlt * iv);
        cr[i] = rec;
    }
    if (hp->overflow) decay_over_super(r, tile, lane, m, e);
    double v[3] = {tau, -m, e};
    wave_max_dpp<3>(v);
    tau = v[0];
    const double lb = hp->lb_build * G * (1.0 - kTiny);
    if (lane == 0) {
        hp->lb_out = lb;
        hp->lbout32 = f32_down(lb);
        if (!hp->overflow) {
            hp->tau = tau * (1.0 + kTiny) + kUnder;
            hp->slack32 = screen_slack32(hp->tau);
        }
    }
    relax_tile_bound(r, tile, lane, f0, -v[1], v[2], lb);
}

template <int D, int PREC, typename RT>
__device__ __forceinline__ void tilecand_body(RT r, const int bid)
{
    const DevState* st = r.st;
    if (round_over(st)) return;
    constexpr int kCpl = 4;   // list entries a lane keeps in registers between passes
    // per wave: the kept candidates (center, squared smallest effective box
    // distance), then in the same slot the candidate's record
    union Slot {
        CandRec rec;
        struct { double lo2; int c; } k;
    };
    __shared__ Slot s_slot[kBlock / kWave][kTileCap];
    __shared__ float s_key[kBlock / kWave][kTileCap];
    const int lane = threadIdx.x % kWave;
    const int wv = threadIdx.x / kWave;
    // wave-uniform: the tile box, its frame and the list bounds live in scalar registers
    const int tile = __builtin_amdgcn_readfirstlane(bid * (kBlock / kWave) + (int)threadIdx.x / kWave);
    if (tile >= r.ntiles) return;
    if (st->lists_ok) {
        // the sweep keeps the lists of the last build
        refresh_tile(r, tile, lane);
        return;
    }
    const TileBound f0 = r.tbnd[tile];
    const int k = r.k;
    const double* __restrict__ C = r.C;

    double blo[D], bhi[D], X[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        blo[j] = r.tbox[(int64_t)tile * 2 * D + j];
        bhi[j] = r.tbox[(int64_t)tile * 2 * D + D + j];
        X[j] = r.tframe[tile].X[j];
    }
    const double Rn = r.tframe[tile].hnorm * (1.0 + kTiny);
    const double pnt = (D == 3 ? kFixPt3 : kFixPt2) * Rn;   // fixed-point term of the bound
    const int sidx = tile / r.super_tiles;
    const int L = r.scount[sidx];
    const int* __restrict__ sl = r.slist + (int64_t)sidx * k;
    CandRec* __restrict__ out = r.tcand + (int64_t)tile * kTileCap;
    const unsigned long long below = (1ULL << lane) - 1ULL;

    // candidates that pass the filter, compacted into the wave's slots
    // (their count goes on beyond kTileCap: the tile then overflows)
    int cnt = 0;
    auto keep_if = [&](bool keep, int c, double lo2) {
        const unsigned long long b = wave_ballot(keep);
        const int pos = cnt + (int)__popcll(b & below);
        if (keep && pos < kTileCap) {
            s_slot[wv][pos].k.lo2 = lo2;
            s_slot[wv][pos].k.c = c;
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
        t = wave_two_dpp(t);
        thr2 = t.b * (1.0 + 2.0 * kCandSlack) * kListMargin2;
#pragma unroll
        for (int u = 0; u < kCpl; ++u)
            if (u * kWave < L) keep_if(cc[u] >= 0 && clo[u] <= thr2, cc[u], clo[u]);
    } else {
        for (int i = lane; i < L; i += kWave) {
            const int c = sl[i];
            double lo2, hi2;
            box_eff2<D>(blo, bhi, C, k, c, r.clus[c].y, lo2, hi2);
            t = merge_two(t, Two{hi2, kInf});
        }
        t = wave_two_dpp(t);
        thr2 = t.b * (1.0 + 2.0 * kCandSlack) * kListMargin2;
        for (int i0 = 0; i0 < L; i0 += kWave) {
            const int i = i0 + lane;
            int c = 0;
            bool keep = false;
            double lo2 = 0.0;
            if (i < L) {
                c = sl[i];
                double hi2;
                box_eff2<D>(blo, bhi, C, k, c, r.clus[c].y, lo2, hi2);
                keep = lo2 <= thr2;
            }
            keep_if(keep, c, lo2);
        }
    }
    // an overflowed tile is swept in FP64 over the super-tile list (its
    // FP32 bounds are not used)
    const bool overflow = cnt > kTileCap;
    const int nrec = min(cnt, kTileCap);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // error bounds of every kept candidate and its record (one lane each,
    // in place of its slot)
    double tau = 0.0, dmax = 0.0, m = 1.0, e = 0.0;
    for (int i = lane; i < nrec; i += kWave) {
        const double lo2 = s_slot[wv][i].k.lo2;
        const int c = s_slot[wv][i].k.c;
        const double iv = r.clus[c].y;
        const double2 dc = r.cdec[c];
        m = fmin(m, dc.x);
        e = fmax(e, dc.y);
        double dd = 0.0, q[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            q[j] = C[(int64_t)j * k + c] - X[j];
            dd += q[j] * q[j];
        }
        const double delta = pnt + 8.0 * kU32 * (Rn + sqrt(dd) * (1.0 + kTiny)) + kUnder;
        const double tc = delta * iv;
        dmax = fmax(dmax, delta);
        tau = fmax(tau, tc);
        const double lk = sqrt(lo2) * (1.0 - 10.0 * kU32) - tc * (1.0 + kTiny);
        CandRec rec;
        rec.qx = (float)q[0];
        rec.qy = (float)q[1];
        rec.qz = D == 3 ? (float)q[D - 1] : 0.0f;
        rec.w2 = screen_w2(iv);
        rec.id = c;
        rec.key = lk > 0.0 ? f32_down(lk * lk * (1.0 - 4.0 * kU32)) : 0.0f;
        rec.dlt = f32_up(delta);
        rec.key0 = rec.key;
        s_slot[wv][i].rec = rec;
        s_key[wv][i] = rec.key;
    }
    if (overflow) decay_over_super(r, tile, lane, m, e);
    {
        double v[4] = {tau, dmax, -m, e};
        wave_max_dpp<4>(v);
        tau = v[0];
        dmax = v[1];
        m = -v[2];
        e = v[3];
    }
    // the records in ascending key order (ties by slot): each lane ranks its
    // records against all of them (the wave's own LDS rows, so a wave-level
    // fence orders the writes before the reads)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (!overflow) {
        for (int i = lane; i < nrec; i += kWave) {
            const float ki = s_key[wv][i];
            int rank = 0;
            for (int j = 0; j < nrec; ++j) {
                const float kj = s_key[wv][j];
                rank += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
            }
            out[rank] = s_slot[wv][i].rec;
        }
    }
    if (lane == 0) {
        const TileFrame& fr = r.tframe[tile];
        TileHead h;
        h.n = overflow ? 0 : cnt;
        h.overflow = overflow ? 1 : 0;
        h.tau = tau * (1.0 + kTiny) + kUnder;
        h.dmax = dmax * (1.0 + kTiny);
        h.lb_out = sqrt(t.b * kListMargin2) * (1.0 - kTiny);
        h.lb_build = h.lb_out;
        h.step[0] = fr.step[0];
        h.step[1] = fr.step[1];
        h.step[2] = fr.step[2];
        h.slack32 = screen_slack32(h.tau);
        h.ubadd32 = f32_up((h.dmax + 2.0 * kSqrtAbs * (1.0 + 7.0 * kU32)) * (1.0 + 0x1p-20));
        h.lbout32 = f32_down(h.lb_out);
        r.thead[tile] = h;
        if (tile == 0) atomicAdd(r.cnt + kCntListBuilds, 1ULL);
    }
    relax_tile_bound(r, tile, lane, f0, m, e, sqrt(t.b * kListMargin2) * (1.0 - kTiny));
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
// block id, stored bounds (one 8-byte record), Hamerly test.  The points the
// bounds cannot decide are compacted into an LDS work list, and phase 2
// gives each of them a full lane for the candidate scan (records staged in
// LDS, in ascending key order, so the scan stops once no later record can
// matter to any lane of the wave), the decision and the block-weight
// bookkeeping, so skipped points cost no candidate arithmetic.  The
// coordinate sums of the center update are not touched here: the round-end
// pass rebuilds them from the final assignment.
//
// FP32 arithmetic of the decision and the stored bounds.  With u = 2^-24 and
// RN the FP32 rounding, every quantity below is rounded in the safe
// direction:
//   * Hamerly test: U = (ub + D) / I, L = M lb - E with the stored ub, lb,
//     the movement D and 1/I rounded up (clus32.x, .y), M rounded down, E
//     up; RN(RN(ub + D) * (1/I)) >= U (1 - u)^2, and RN(M lb - E) (one
//     fused multiply-add) <= L (1 + u) when positive; the point is skipped
//     when RN(ubf (1 + 2^-20) + 2^-100) < lbf, which then implies U < L.
//   * sure decision: with kM <= 1 - kScr - 4u and kP >= 1 + kScr + 4u,
//     RN(es kM - eb kP) > 2 slack32 implies the exact-arithmetic test
//     es (1 - kScr) - eb (1 + kScr) > 2 slack (slack32 >= slack, the
//     rounding of es kM and of the fused difference is within the 4u).
//   * bounds of a sure point: RN(sqrt_raw(d2) (1 + 10u) + ubadd32) >= the
//     FP64 form (sqrt_raw(d2) + 2^-46)(1 + 7u) + dmax; RN(es kM - slack32)
//     <= es (1 - kScr) - slack for both signs of the result.
//   * stored upper bound: t = RN(ubf - Ddn) with the movement rounded down
//     (clusdn);
//     RN(|t| 2^-22 + (t + 2^-120)) >= ubf - Ddn.
//   * stored lower bound: RN(RN(lbf + Edn) invMdn) <= (lb + E) / M when
//     lbf + Edn >= 0 (Edn <= E, invMdn <= (1 - 2^-22) / M); a negative
//     value is stored as 0, which is always valid.
// FP64 results (recheck, plain FP64 sweep) enter the same stores through
// f32_up_q / f32_dn_q: RN(RN(x)(1 + 2^-22) + 2^-120) >= x and, for x >= 0,
// RN(RN(x)(1 - 2^-22)) <= x (flushed to 0 below 2^-100).
__device__ inline float f32_up_q(double x)
{
    return __builtin_fmaf((float)x, 1.0f + 0x1p-22f, 0x1p-120f);
}

__device__ inline float f32_dn_q(double x)
{
    const float y = (float)x * (1.0f - 0x1p-22f);
    return y < 0x1p-100f ? 0.0f : y;
}

constexpr float kM32 = 1.0f - 15.0f * 0x1p-24f;   // <= 1 - kScr - 4u
constexpr float kP32 = 1.0f + 16.0f * 0x1p-24f;   // >= 1 + kScr + 4u
constexpr float kUb32 = 1.0f + 10.0f * 0x1p-24f;  // 1 + 10u

template <int D, int PREC, int PPT, bool WEIGHTED, typename RT>
__device__ __forceinline__ void sweep_body(RT r, const int bid)
{
    DevState* st = r.st;
    if (round_over(st)) return;
    constexpr bool F32 = PREC == BKM_PREC_F32_RECHECK;
    constexpr int T = kBlock * PPT;
    __shared__ int s_off[T];      // tile offsets of the points to evaluate
    __shared__ int s_aold[T];     // and their current block
    __shared__ int s_gflag[T / kWave];  // per 64-point group: common block, or -1
    __shared__ int s_gdirty[T / kWave]; // per 64-point group: a point of it changed block
    __shared__ float4 s_q[kTileCap];
    __shared__ float s_key[kTileCap];
    __shared__ int s_cid[kTileCap];
    __shared__ double s_c64[4][kTileCap];   // FP64 centers and (1/I)^2 (FP64 sweep, overflow)
    __shared__ int s_nl;
    __shared__ unsigned long long s_cnt[kBlock / kWave][5];   // counters of each wave

    const int tid = threadIdx.x, lane = tid % kWave;
    const int tile = bid;
    const int64_t base = (int64_t)tile * T;
    const int k = r.k;
    const double* __restrict__ C = r.C;
    const double* __restrict__ I = r.I;
    // per-tile views: a 32-bit offset from a wave-uniform base per access
    int32_t* __restrict__ At = r.A + base;
    float2* __restrict__ Bt = r.bnd + base;
    if (tid == 0) s_nl = 0;
    if (tid < T / kWave) s_gdirty[tid] = 0;

    // ---- phase 1: block ids and stored bounds (arrays are padded to whole tiles)
    int aold[PPT];
    float2 bd[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const unsigned i = (unsigned)(q * kBlock + tid);
        aold[q] = At[i];
        bd[q] = Bt[i];
    }
    const TileHead hd = r.thead[tile];
    const int sidx = tile / r.super_tiles;
    const int* __restrict__ sl = r.slist + (int64_t)sidx * k;
    const CandRec* __restrict__ cr = r.tcand + (int64_t)tile * kTileCap;
    const int ncand = hd.overflow ? r.scount[sidx] : hd.n;
    // the tile's candidate records into LDS; an odd count is padded with a
    // record no point can pick (its values are +inf), so the scan can take
    // the records two at a time
    if (!hd.overflow && tid <= hd.n) {
        if (tid < hd.n) {
            const CandRec rec = cr[tid];
            s_cid[tid] = rec.id;
            s_key[tid] = rec.key;
            if (F32) {
                s_q[tid] = make_float4(rec.qx, rec.qy, rec.qz, rec.w2);
            } else {
                const double iv = r.clus[rec.id].y;
                s_c64[0][tid] = C[rec.id];
                s_c64[1][tid] = C[(int64_t)k + rec.id];
                s_c64[2][tid] = D == 3 ? C[(int64_t)(D - 1) * k + rec.id] : 0.0;
                s_c64[3][tid] = iv * iv;
            }
        } else if ((hd.n & 1) && tid < kTileCap) {
            s_cid[tid] = 0;
            s_key[tid] = INFINITY;
            s_q[tid] = make_float4(0x1p120f, 0x1p120f, 0x1p120f, 1.0f);
            s_c64[0][tid] = s_c64[1][tid] = s_c64[2][tid] = 0x1p600;
            s_c64[3][tid] = 1.0;
        }
    }
    float2 cl[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) cl[q] = r.clus32[aold[q] > 0 ? aold[q] : 0];
    // the tile's lower-bound frame in FP32, rounded so that every bound
    // stays valid; without bounds the test below can never pass (its lower
    // bound is -inf)
    const TileBound tb = r.tbnd[tile];
    const float Mf = r.use_bounds ? tb.Mf : 0.0f;
    const float Ef = r.use_bounds ? tb.Ef : INFINITY;
    const float Edn = tb.Edn, invMdn = tb.invMdn, lam = tb.lam;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    // Hamerly test (Sec. 4.3) of every point: upper bound on the own
    // effective distance below the lower bound on the second-best one (a
    // point without a block yet has an infinite upper bound)
    unsigned long long bq[PPT];
    unsigned n_eval = 0, n_skip = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const bool real = aold[q] != kPad && ncand > 0;
        const float ub = (bd[q].x + cl[q].x) * cl[q].y;
        // the stored bound, lowered to the tile's floor for the centers
        // left out of its list (a skipped point keeps the lowered value)
        const float sq = fminf(bd[q].y, lam);
        const float lb = __builtin_fmaf(Mf, sq, -Ef);
        const bool skip = __builtin_fmaf(ub, 1.0f + 0x1p-20f, 0x1p-100f) < lb;
        if (real && skip && sq < bd[q].y) Bt[q * kBlock + tid].y = sq;
        bq[q] = wave_ballot(real & !skip);
        const unsigned nr = (unsigned)__popcll(wave_ballot(real));
        const unsigned ne = (unsigned)__popcll(bq[q]);
        n_eval += ne;
        n_skip += nr - ne;
    }
    // one LDS reservation per wave for all its points to evaluate
    __syncthreads();   // s_nl initialised
    int run = 0;
    if (lane == 0 && n_eval) run = atomicAdd(&s_nl, (int)n_eval);
    run = __builtin_amdgcn_readfirstlane(run);
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        if ((bq[q] >> lane) & 1ULL) {
            const int pos = run + (int)__popcll(bq[q] & below);
            s_off[pos] = q * kBlock + tid;
            s_aold[pos] = aold[q];
        }
        run += (int)__popcll(bq[q]);
        // the wave holds one whole 64-point group here: its common block
        const int a0 = __builtin_amdgcn_readfirstlane(aold[q]);
        const bool same = wave_ballot(aold[q] != a0) == 0ULL;
        if (lane == 0) s_gflag[q * (kBlock / kWave) + tid / kWave] = same ? a0 : -1;
    }
    __syncthreads();
    const int nl = s_nl;

    // ---- phase 2: one lane per undecided point
    unsigned n_rechk = 0, n_chg = 0, n_bad = 0;
    unsigned long long n_cand = 0;
    const float gap32 = (float)r.recheck_gap;
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
        const unsigned nact = (unsigned)__popcll(wave_ballot(act));
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
        // the ranking by squared effective distance s * (1/I)^2, iv2 = (1/I)^2,
        // ties to the lower center index.  Its rounding differs from
        // sqrt(s) / I by a few units of 2^-53, which can only swap two
        // candidates closer than that (a tie at the 1e-12 level), and the
        // bounds below carry a 1e-12 slack.
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
        if (!hd.overflow) {
            if (nact) {
                // records in ascending key order, taken two at a time: stop
                // once every active lane's second-best value is at most the
                // next key -- no later record can change its best or
                // second-best (for FP64 the key is strictly above it)
                int c0 = 0;
                for (; c0 < ncand; c0 += 2) {
                    const float key = s_key[c0];
                    if (F32) {
                        if (wave_ballot(act & (s2 > key)) == 0ULL) break;
                        const float4 qa = s_q[c0];
                        const float4 qb = s_q[c0 + 1];
                        consider32(c0, qa.x, qa.y, qa.z, qa.w);
                        consider32(c0 + 1, qb.x, qb.y, qb.z, qb.w);
                    } else {
                        if (wave_ballot(act & !(se < (double)key)) == 0ULL) break;
                        consider64sq(s_cid[c0], s_c64[0][c0], s_c64[1][c0], s_c64[2][c0],
                                     s_c64[3][c0]);
                        if (c0 + 1 < ncand)
                            consider64sq(s_cid[c0 + 1], s_c64[0][c0 + 1], s_c64[1][c0 + 1],
                                         s_c64[2][c0 + 1], s_c64[3][c0 + 1]);
                    }
                }
                n_cand += (unsigned long long)nact * (unsigned)min(c0, ncand);
            }
            if (!F32) se = sqrt(se);
        } else {
            // overflowed tile: the super-tile's list in FP64, staged through
            // LDS in chunks of kTileCap centers that every wave of the block
            // helps to load (the loop is block-uniform)
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
                if (nact) {
                    for (int c0 = 0; c0 < m; ++c0)
                        consider64sq(s_cid[c0], s_c64[0][c0], s_c64[1][c0], s_c64[2][c0], s_c64[3][c0]);
                }
            }
            n_cand += (unsigned long long)nact * (unsigned)ncand;
            // back to effective distances for the lower bound
            se = sqrt(se);
        }
        int cbest = ao;
        bool chg = false, rck = false, bad = false;
        long long wh = 1, wl = 0;
        if (act) {
            float ubf, lbf;   // upper bound on the own distance, lower bound on the second-best
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
                const float eb = sqrt_raw(be2);
                const float es = sqrt_raw(s2);
                const float sl32 = hd.slack32;
                // one candidate: certain; an overflowed FP32 value: decide in FP64
                const bool sure =
                    b2 < INFINITY &&
                    (ncand == 1 ||
                     (s2 < INFINITY && __builtin_fmaf(-eb, kP32, es * kM32) > 2.0f * sl32 &&
                      es - eb > gap32 * es));
                if (sure) {
                    cbest = bc;
                    ubf = __builtin_fmaf(sqrt_raw(bd2), kUb32, hd.ubadd32);
                    lbf = __builtin_fmaf(es, kM32, -sl32);
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
                    const double slack = hd.tau * (1.0 + 16.0 * kU32) + 2.0 * kSqrtAbs;
                    const double win = (double)eb * (1.0 + kScr) + 2.0 * slack;
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
                    ubf = f32_up_q(sqrt(bsq) * (1.0 + kTiny));
                    lbf = f32_dn_q(fmin(s, win - slack) * (1.0 - kTiny));
                }
            } else {
                cbest = bc;
                ubf = f32_up_q(sqrt(bs2) * (1.0 + kTiny));
                lbf = f32_dn_q(se * (1.0 - kTiny));
            }
            // a decision without a valid block is an internal error: it is
            // counted (the call then fails) and the point keeps a valid block
            if (cbest < 0 || cbest >= k) {
                bad = true;
                cbest = ao >= 0 ? ao : 0;
            }
            lbf = fminf(lbf, hd.lbout32);
            {
                const float t = ubf - r.clusdn[cbest];
                const float ut = __builtin_fmaf(fabsf(t), 0x1p-22f, t + 0x1p-120f);
                const float lt = (lbf + Edn) * invMdn;
                Bt[off] = make_float2(ut, fmaxf(lt, 0.0f));
            }
            if (cbest != ao) {
                chg = true;
                At[off] = cbest;
                s_gflag[off / kWave] = -1;   // conservatively mixed from now on
                s_gdirty[off / kWave] = 1;
                if (WEIGHTED) fix_split(r.ws[p] * wsc, wh, wl);
            }
        }
        n_rechk += (unsigned)__popcll(wave_ballot(rck));
        n_bad += (unsigned)__popcll(wave_ballot(bad));
        // wave-aggregated transfer of the point's weight from the old to the new block
        unsigned long long pend = wave_ballot(chg);
        n_chg += (unsigned)__popcll(pend);
        while (pend) {
            const int leader = __builtin_ctzll(pend);
            const int ka = __shfl(ao, leader, kWave);
            const int kb = __shfl(cbest, leader, kWave);
            const bool mine = chg && ao == ka && cbest == kb;
            const unsigned long long mm = wave_ballot(mine);
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
        s_cnt[wv][4] = n_cand;
        if (n_bad) {
            unsigned long long* slot = r.cnt + (int64_t)(tile % kCntSlots) * kCntWords;
            atomicAdd(slot + kCntInvalid, (unsigned long long)n_bad);
        }
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
