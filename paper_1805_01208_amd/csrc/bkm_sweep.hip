// Assignment sweep of balanced k-means (Alg. 1 inner loop; Sec. 4.2-4.4).
//
// Every point takes the center with the smallest effective distance
// dist(p, c) / influence(c).  Two exact prunings from the paper, laid out for
// the GPU:
//   * centers (Sec. 4.4): for a box B of points, a center whose smallest
//     possible effective distance to B exceeds the second-smallest largest
//     effective distance of any center to B can be neither the best nor the
//     second-best center of any point in B.  The filter runs at two levels:
//     super-tiles against all k centers (k_supercand), then each tile of
//     consecutive Hilbert-ordered points against its super-tile's list, inside
//     the sweep block, into LDS.
//   * points (Sec. 4.3, Hamerly): a point whose upper bound on the effective
//     distance to its own center is below its lower bound on the second-best
//     effective distance keeps its block without evaluating anything.  The
//     bounds are stored lazily -- the upper bound as a distance relative to the
//     accumulated movement of its center, the lower bound in a global affine
//     frame (M, E) -- so a point that is skipped is never written.
// Block weights and the weighted coordinate sums of the center update are
// maintained incrementally: a point that changes block moves its exact
// fixed-point terms from the old to the new block with integer atomics, so the
// sums equal the from-scratch sums bit for bit and do not depend on
// scheduling order.
#include <math.h>

#include "bkm_internal.h"

namespace bkm {

namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24, unit roundoff of FP32
constexpr double kCandSlack = 1e-9;               // relative slack of the center filter
constexpr double kTiny = 1e-12;                   // relative slack of FP64 bound arithmetic
constexpr double kInf = INFINITY;

// Smallest and largest effective distance from center c to the box [lo, hi].
template <int D>
__device__ inline void box_eff(const double* lo, const double* hi, const double* C, int k,
                               int c, double infl, double& lo_eff, double& hi_eff)
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
    lo_eff = sqrt(mn) / infl;
    hi_eff = sqrt(mx) / infl;
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

template <int D>
__global__ __launch_bounds__(kBlock) void k_supercand(RunDev r)
{
    const DevState* st = r.st;
    if (st->done || st->round_done) return;
    __shared__ double sa[kBlock / kWave], sb[kBlock / kWave];
    __shared__ int cnt;
    const int s = blockIdx.x, tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int k = r.k;
    double lo[D], hi[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lo[j] = r.sbox[(int64_t)s * 2 * D + j];
        hi[j] = r.sbox[(int64_t)s * 2 * D + D + j];
    }
    Two t{kInf, kInf};
    for (int c = tid; c < k; c += kBlock) {
        double le, he;
        box_eff<D>(lo, hi, r.C, k, c, r.I[c], le, he);
        t = merge_two(t, Two{he, kInf});
    }
    t = wave_two(t);
    if (lane == 0) {
        sa[wv] = t.a;
        sb[wv] = t.b;
    }
    if (tid == 0) cnt = 0;
    __syncthreads();
    Two all{sa[0], sb[0]};
    for (int w = 1; w < kBlock / kWave; ++w) all = merge_two(all, Two{sa[w], sb[w]});
    const double thr = all.b * (1.0 + kCandSlack);
    int* out = r.slist + (int64_t)s * k;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    for (int c0 = 0; c0 < k; c0 += kBlock) {
        const int c = c0 + tid;
        bool keep = false;
        if (c < k) {
            double le, he;
            box_eff<D>(lo, hi, r.C, k, c, r.I[c], le, he);
            keep = le <= thr;
        }
        const unsigned long long b = __ballot(keep);
        int off = 0;
        if (lane == 0 && b) off = atomicAdd(&cnt, (int)__popcll(b));
        off = __shfl(off, 0, kWave);
        if (keep) out[off + __popcll(b & below)] = c;
    }
    __syncthreads();
    if (tid == 0) r.scount[s] = cnt;
}

// One sweep.  Block = one tile of T = 256 * PPT consecutive Hilbert-ordered
// points; thread t handles points base + t + 256 q, so each wave covers
// 64-point groups and every global access is coalesced.
template <int D, int PREC, int PPT, bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_sweep(RunDev r)
{
    DevState* st = r.st;
    if (st->done || st->round_done) return;
    constexpr bool F32 = PREC == BKM_PREC_F32_RECHECK;

    __shared__ double s_lo[kLcap];
    __shared__ int s_id[kMaxc];
    __shared__ int s_cid[kMaxc];
    __shared__ float s_q[D][kMaxc];
    __shared__ float s_w2[kMaxc];
    __shared__ double s_c[F32 ? 1 : D][F32 ? 1 : kMaxc];
    __shared__ double s_I[F32 ? 1 : kMaxc];
    __shared__ double s_red[2 * (kBlock / kWave)];
    __shared__ int s_nc;
    __shared__ unsigned long long s_cnt[5];

    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    const int tile = blockIdx.x;
    const int64_t base = (int64_t)tile * r.T;
    const int k = r.k;
    const double* __restrict__ C = r.C;
    const double* __restrict__ I = r.I;

    // tile geometry: exact box, anchor X (box center), half-extent norm
    double blo[D], bhi[D], X[D];
    double rn2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        blo[j] = r.tbox[(int64_t)tile * 2 * D + j];
        bhi[j] = r.tbox[(int64_t)tile * 2 * D + D + j];
        X[j] = 0.5 * (blo[j] + bhi[j]);
        const double h = fmax(bhi[j] - X[j], X[j] - blo[j]);
        rn2 += h * h;
    }
    const double Rn = sqrt(rn2) * (1.0 + kTiny);

    // tile-level center filter over the super-tile's candidates
    const int sidx = tile / r.super_tiles;
    const int L = r.scount[sidx];
    const int* sl = r.slist + (int64_t)sidx * k;
    Two t{kInf, kInf};
    for (int i = tid; i < L; i += kBlock) {
        const int c = sl[i];
        double le, he;
        box_eff<D>(blo, bhi, C, k, c, I[c], le, he);
        if (i < kLcap) s_lo[i] = le;
        t = merge_two(t, Two{he, kInf});
    }
    t = wave_two(t);
    if (lane == 0) {
        s_red[wv] = t.a;
        s_red[kBlock / kWave + wv] = t.b;
    }
    if (tid < 5) s_cnt[tid] = 0;
    if (tid == 0) s_nc = 0;
    __syncthreads();
    Two all{s_red[0], s_red[kBlock / kWave]};
    for (int w = 1; w < kBlock / kWave; ++w) all = merge_two(all, Two{s_red[w], s_red[kBlock / kWave + w]});
    const double thr = all.b * (1.0 + kCandSlack);
    bool overflow = L > kLcap;
    if (!overflow) {
        const unsigned long long below = (1ULL << lane) - 1ULL;
        for (int i0 = 0; i0 < L; i0 += kBlock) {
            const int i = i0 + tid;
            const bool keep = i < L && s_lo[i] <= thr;
            const unsigned long long b = __ballot(keep);
            int off = 0;
            if (lane == 0 && b) off = atomicAdd(&s_nc, (int)__popcll(b));
            off = __shfl(off, 0, kWave);
            const int pos = off + (int)__popcll(b & below);
            if (keep && pos < kMaxc) s_id[pos] = sl[i];
        }
    }
    __syncthreads();
    if (!overflow && s_nc > kMaxc) overflow = true;
    const int* src = overflow ? sl : s_id;
    const int ncand = overflow ? L : s_nc;
    // a lower bound on the effective distance of every center left out
    const double lb_out = thr * (1.0 - kTiny);

    // FP32 error constants of this tile (see the sweep notes below)
    double tau = 0.0, dmax = 0.0;
    if (F32) {
        for (int i = tid; i < ncand; i += kBlock) {
            const int c = src[i];
            double dd = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double v = C[(int64_t)j * k + c] - X[j];
                dd += v * v;
            }
            const double delta = 8.0 * kU32 * (Rn + sqrt(dd) * (1.0 + kTiny));
            dmax = fmax(dmax, delta);
            tau = fmax(tau, delta / I[c]);
        }
        tau = wave_max_d(tau);
        dmax = wave_max_d(dmax);
        if (lane == 0) {
            s_red[wv] = tau;
            s_red[kBlock / kWave + wv] = dmax;
        }
        __syncthreads();
        tau = s_red[0];
        dmax = s_red[kBlock / kWave];
        for (int w = 1; w < kBlock / kWave; ++w) {
            tau = fmax(tau, s_red[w]);
            dmax = fmax(dmax, s_red[kBlock / kWave + w]);
        }
        tau *= 1.0 + kTiny;
        dmax *= 1.0 + kTiny;
    }

    // load points, Hamerly test
    const double M = st->M, E = st->E;
    int aold[PPT];
    bool ev[PPT];
    float o[PPT][D];
    double x[PPT][D];
    float b2[PPT], s2[PPT], bd2[PPT];
    int bi[PPT];
    double be[PPT], se[PPT], bs2[PPT];
    int bc[PPT];
    unsigned n_eval = 0, n_skip = 0;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * kBlock + tid;
        const bool valid = p < r.n;
        aold[q] = valid ? r.A[p] : -1;
        ev[q] = valid;
        if (valid && r.use_bounds && aold[q] >= 0) {
            const double2 cl = r.clus[aold[q]];
            const double ub = ((double)r.ubt[p] + cl.x) * cl.y * (1.0 + kTiny);
            const double lt = (double)r.lbt[p];
            const double lb = (M * lt - E) - kTiny * (M * lt + E);
            if (ub < lb) {
                ev[q] = false;
                ++n_skip;
            }
        }
        if (ncand == 0) ev[q] = false;  // no candidate (cannot happen for finite data)
        if (ev[q]) ++n_eval;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            o[q][j] = 0.0f;
            x[q][j] = 0.0;
            if (ev[q]) {
                if (F32)
                    o[q][j] = r.ofs[j][p];
                else
                    x[q][j] = sorted_coord(r, j, p);
            }
        }
        b2[q] = s2[q] = bd2[q] = INFINITY;
        bi[q] = 0;
        be[q] = se[q] = bs2[q] = kInf;
        bc[q] = 0x7fffffff;
    }
    bool anyev = false;
#pragma unroll
    for (int q = 0; q < PPT; ++q) anyev |= ev[q];
    const bool wave_busy = __ballot(anyev) != 0ULL;

    // evaluate the candidates, chunk by chunk through LDS
    for (int cs = 0; cs < ncand; cs += kMaxc) {
        const int cn = min(kMaxc, ncand - cs);
        __syncthreads();
        for (int i = tid; i < cn; i += kBlock) {
            const int c = src[cs + i];
            s_cid[i] = c;
            if (F32) {
#pragma unroll
                for (int j = 0; j < D; ++j) s_q[j][i] = (float)(C[(int64_t)j * k + c] - X[j]);
                const float iv = (float)(1.0 / I[c]);
                s_w2[i] = iv * iv;
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) s_c[F32 ? 0 : j][F32 ? 0 : i] = C[(int64_t)j * k + c];
                s_I[F32 ? 0 : i] = I[c];
            }
        }
        __syncthreads();
        if (!wave_busy) continue;
        for (int i = 0; i < cn; ++i) {
            if (F32) {
                const float q0 = s_q[0][i], q1 = s_q[1][i], q2 = D == 3 ? s_q[D - 1][i] : 0.0f;
                const float w2 = s_w2[i];
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    const float dx = o[q][0] - q0;
                    const float dy = o[q][1] - q1;
                    float d2 = dx * dx;
                    d2 = __builtin_fmaf(dy, dy, d2);
                    if (D == 3) {
                        const float dz = o[q][D - 1] - q2;
                        d2 = __builtin_fmaf(dz, dz, d2);
                    }
                    const float e2 = d2 * w2;
                    if (e2 < b2[q]) {
                        s2[q] = b2[q];
                        b2[q] = e2;
                        bd2[q] = d2;
                        bi[q] = cs + i;
                    } else if (e2 < s2[q]) {
                        s2[q] = e2;
                    }
                }
            } else {
                const int c = s_cid[i];
                const double cx = s_c[0][F32 ? 0 : i], cy = s_c[F32 ? 0 : 1][F32 ? 0 : i];
                const double cz = D == 3 ? s_c[F32 ? 0 : D - 1][F32 ? 0 : i] : 0.0;
                const double ic = s_I[F32 ? 0 : i];
#pragma unroll
                for (int q = 0; q < PPT; ++q) {
                    double sq;
                    const double e = eff64<D>(x[q], cx, cy, cz, ic, sq);
                    if (e < be[q] || (e == be[q] && c < bc[q])) {
                        se[q] = be[q];
                        be[q] = e;
                        bc[q] = c;
                        bs2[q] = sq;
                    } else if (e < se[q]) {
                        se[q] = e;
                    }
                }
            }
        }
    }

    // decide, store bounds, move fixed-point terms of points that changed block
    unsigned n_rechk = 0, n_chg = 0;
    const double gap_rel = r.recheck_gap;
    const double lo0 = st->lo[0], lo1 = st->lo[1], lo2 = st->lo[D - 1];
    const double sxs = st->sx_scale, wsc = st->w_scale;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int64_t p = base + (int64_t)q * kBlock + tid;
        int cbest = aold[q];
        bool chg = false;
        long long th[D], tl[D], wh = 1, wl = 0;
        if (ev[q]) {
            double ubd, lb;
            bool have64 = !F32;
            if (F32) {
                const float eb = __builtin_sqrtf(b2[q]);
                const float es = __builtin_sqrtf(s2[q]);
                // single candidate: certain; an overflowed FP32 value: decide in FP64
                const bool sure =
                    b2[q] < INFINITY &&
                    (ncand == 1 ||
                     (s2[q] < INFINITY &&
                      (double)es * (1.0 - 8.0 * kU32) - (double)eb * (1.0 + 8.0 * kU32) > 2.0 * tau &&
                      (double)es - (double)eb > gap_rel * (double)es));
                if (sure) {
                    cbest = src[bi[q]];
                    ubd = (double)__builtin_sqrtf(bd2[q]) * (1.0 + 4.0 * kU32) + dmax;
                    lb = (double)es * (1.0 - 8.0 * kU32) - tau;
                } else {
                    // FP64 recheck over every candidate of the tile
                    ++n_rechk;
#pragma unroll
                    for (int j = 0; j < D; ++j) x[q][j] = sorted_coord(r, j, p);
                    have64 = true;
                    double b = kInf, s = kInf, bsq = kInf;
                    int bcc = 0x7fffffff;
                    for (int i = 0; i < ncand; ++i) {
                        const int c = src[i];
                        double sq;
                        const double e = eff64<D>(x[q], C[c], C[(int64_t)k + c],
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
                    lb = s * (1.0 - kTiny);
                }
            } else {
                cbest = bc[q];
                ubd = sqrt(bs2[q]) * (1.0 + kTiny);
                lb = se[q] * (1.0 - kTiny);
            }
            if (cbest < 0 || cbest >= k) cbest = aold[q] >= 0 ? aold[q] : src[0];
            lb = fmin(lb, lb_out);
            if (r.use_bounds) {
                const double Db = r.clus[cbest].x;
                double uv = ubd - Db;
                uv += kTiny * (fabs(ubd) + Db);
                r.ubt[p] = f32_up(uv);
                double lv = (lb + E) / M;
                lv -= kTiny * fabs(lv);
                r.lbt[p] = (lv > 0.0) ? f32_down(lv) : 0.0f;
            }
            if (cbest != aold[q]) {
                chg = true;
                ++n_chg;
                r.A[p] = cbest;
                if (!have64) {
#pragma unroll
                    for (int j = 0; j < D; ++j) x[q][j] = sorted_coord(r, j, p);
                }
                const double w = WEIGHTED ? r.ws[p] : 1.0;
                const double lov[3] = {lo0, lo1, lo2};
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    double v = x[q][j] - lov[j];
                    if (WEIGHTED) v = w * v;
                    fix_split(v * sxs, th[j], tl[j]);
                }
                if (WEIGHTED) fix_split(w * wsc, wh, wl);
            }
        }
        // wave-aggregated transfer of the terms from the old to the new block
        unsigned long long pend = __ballot(chg);
        while (pend) {
            const int leader = (int)__ffsll((long long)pend) - 1;
            const int ka = __shfl(aold[q], leader, kWave);
            const int kb = __shfl(cbest, leader, kWave);
            const bool mine = chg && aold[q] == ka && cbest == kb;
            const unsigned long long mm = __ballot(mine);
            long long v[kAcc];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                v[2 * j] = wave_sum_ll(mine ? th[j] : 0);
                v[2 * j + 1] = wave_sum_ll(mine ? tl[j] : 0);
            }
            if (WEIGHTED) {
                v[6] = wave_sum_ll(mine ? wh : 0);
                v[7] = wave_sum_ll(mine ? wl : 0);
            } else {
                v[6] = (long long)__popcll(mm);
                v[7] = 0;
            }
            if (lane == leader) {
                unsigned long long* nb = (unsigned long long*)(r.acc + (int64_t)kb * kAcc);
                unsigned long long* ob = (unsigned long long*)(r.acc + (int64_t)ka * kAcc);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    atomicAdd(nb + 2 * j, (unsigned long long)v[2 * j]);
                    atomicAdd(nb + 2 * j + 1, (unsigned long long)v[2 * j + 1]);
                    if (ka >= 0) {
                        atomicAdd(ob + 2 * j, (unsigned long long)(-v[2 * j]));
                        atomicAdd(ob + 2 * j + 1, (unsigned long long)(-v[2 * j + 1]));
                    }
                }
                atomicAdd(nb + 6, (unsigned long long)v[6]);
                if (ka >= 0) atomicAdd(ob + 6, (unsigned long long)(-v[6]));
                if (WEIGHTED) {
                    atomicAdd(nb + 7, (unsigned long long)v[7]);
                    if (ka >= 0) atomicAdd(ob + 7, (unsigned long long)(-v[7]));
                }
            }
            pend &= ~mm;
        }
    }

    // counters
    const unsigned long long cev = (unsigned long long)n_eval * (unsigned long long)ncand;
    if (n_eval) atomicAdd(&s_cnt[0], (unsigned long long)n_eval);
    if (n_skip) atomicAdd(&s_cnt[1], (unsigned long long)n_skip);
    if (n_rechk) atomicAdd(&s_cnt[2], (unsigned long long)n_rechk);
    if (n_chg) atomicAdd(&s_cnt[3], (unsigned long long)n_chg);
    if (cev) atomicAdd(&s_cnt[4], cev);
    __syncthreads();
    if (tid == 0) {
        if (s_cnt[0]) atomicAdd(&st->evaluated, s_cnt[0]);
        if (s_cnt[1]) atomicAdd(&st->skipped, s_cnt[1]);
        if (s_cnt[2]) atomicAdd(&st->rechecked, s_cnt[2]);
        if (s_cnt[3]) atomicAdd(&st->changed, s_cnt[3]);
        if (s_cnt[4]) atomicAdd(&st->cand_evals, s_cnt[4]);
        if (overflow) atomicAdd(&st->overflow_tiles, 1ULL);
    }
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
    if (r.d == 2)
        k_supercand<2><<<r.nsuper, kBlock, 0, s>>>(r);
    else
        k_supercand<3><<<r.nsuper, kBlock, 0, s>>>(r);
    return hipGetLastError();
}

hipError_t launch_sweep(const RunDev& r, hipStream_t s)
{
    return r.d == 2 ? sweep_p<2>(r, s) : sweep_p<3>(r, s);
}

}  // namespace bkm
