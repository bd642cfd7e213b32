// k-length updates of balanced k-means and the per-round passes:
//   * balance test and influence adaptation after every sweep (Alg. 1 after
//     the block sizes; Eq. 1 read so that oversized blocks lose influence,
//     clamped to a 5% change per step, Sec. 4.2);
//   * exact per-block bounding boxes of each round's final assignment, for
//     beta, the average cluster diameter of the erosion (Sec. 4.2);
//   * center movement to the weighted block means, the convergence test and
//     the influence erosion (Alg. 2; Sec. 4.2), and the bound relaxation of
//     Eqs. (2)-(3) folded into the lazy bound frames;
//   * run initialisation, outputs, and partition statistics.
#include <math.h>

#include "bkm_internal.h"

namespace bkm {

namespace {

constexpr double kUp = 1.0 + 0x1p-50;     // conservative rounding of bound frames
constexpr double kDown = 1.0 - 0x1p-50;

__device__ inline double block_weight(const RunDev& r, int c)
{
    const long long* a = r.acc + (int64_t)c * kAcc;
    if (!r.weighted) return (double)a[6];
    return fix_value(a[6], a[7]) / r.st->w_scale;
}

// Block-wide reductions for 1024-thread single-block kernels.
template <typename F>
__device__ inline double block_reduce_1024(double v, double* sh, F op)
{
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int m = kWave / 2; m > 0; m >>= 1) v = op(v, __shfl_xor(v, m, kWave));
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = sh[0];
    for (int w = 1; w < 1024 / kWave; ++w) r = op(r, sh[w]);
    return r;
}

// Three reductions at once (the first two minima, the third a maximum).
__device__ inline void block_min_min_max_1024(double& a, double& b, double& c, double (*sh)[1024 / kWave])
{
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int m = kWave / 2; m > 0; m >>= 1) {
        a = fmin(a, __shfl_xor(a, m, kWave));
        b = fmin(b, __shfl_xor(b, m, kWave));
        c = fmax(c, __shfl_xor(c, m, kWave));
    }
    __syncthreads();
    if (lane == 0) {
        sh[0][wv] = a;
        sh[1][wv] = b;
        sh[2][wv] = c;
    }
    __syncthreads();
    a = sh[0][0];
    b = sh[1][0];
    c = sh[2][0];
    for (int w = 1; w < 1024 / kWave; ++w) {
        a = fmin(a, sh[0][w]);
        b = fmin(b, sh[1][w]);
        c = fmax(c, sh[2][w]);
    }
}

struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpAdd { __device__ double operator()(double a, double b) const { return a + b; } };

template <int D, typename RT>
__device__ __forceinline__ void balance_body(RT r, const int bid)
{
    DevState* st = r.st;
    if (round_over(st)) return;
    __shared__ double sh[1024 / kWave];
    const int k = r.k;
    const bool per_block = r.tsz != nullptr;
    double mx = -INFINITY, over = 0.0, ratio = -INFINITY;
    for (int c = threadIdx.x; c < k; c += 1024) {
        const double b = block_weight(r, c);
        mx = fmax(mx, b);
        if (per_block) {
            if (b > r.tL[c]) over = 1.0;
            ratio = fmax(ratio, b / r.tT[c]);
        }
    }
    mx = block_reduce_1024(mx, sh, OpMax());
    if (per_block) {
        over = block_reduce_1024(over, sh, OpMax());
        ratio = block_reduce_1024(ratio, sh, OpMax());
    }
    // balanced: every block within its limit (one common limit, or its own)
    const bool bal = per_block ? over == 0.0 : mx <= st->lmax;
    const int sweep_no = st->sweep_in_round + 1;
    double mu = 1.0, lg = 1.0, lf = 1.0;
    if (!bal) {
        // m: smallest ratio old/new influence (the lower-bound frame); qlo,
        // qhi: smallest and largest ratio of 1/influence to its value at the
        // last candidate-list build
        double m = INFINITY, qlo = INFINITY, qhi = 0.0;
        for (int c = threadIdx.x; c < k; c += 1024) {
            const double s = block_weight(r, c);
            double f;
            if (s > 0.0) {
                const double g = (per_block ? r.tT[c] : st->target) / s;
                f = D == 2 ? sqrt(g) : cbrt(g);
                if (f > 1.05) f = 1.05;
                if (f < 0.95) f = 0.95;
            } else {
                f = 1.05;
            }
            const double io = r.I[c];
            const double in = io * f;
            const double iv = 1.0 / in;
            r.I[c] = in;
            r.clus[c].y = iv;
            r.clus32[c].y = f32_up(iv);
            m = fmin(m, io / in);
            const double q = iv / r.ivb[c];
            qlo = fmin(qlo, q);
            qhi = fmax(qhi, q);
            r.cdec[c] = make_double2(io / in, 0.0);
        }
        __shared__ double sh3[3][1024 / kWave];
        block_min_min_max_1024(m, qlo, qhi, sh3);
        mu = m;
        lg = qlo * kDown;
        lf = qhi * kUp;
    }
    if (bal)
        for (int c = threadIdx.x; c < k; c += 1024) r.cdec[c] = make_double2(1.0, 0.0);
    __syncthreads();
    if (threadIdx.x == 0) {
        st->imu = mu;
        st->ie = 0.0;
        st->sweep_in_round = sweep_no;
        st->sweeps += 1;
        st->balanced = bal ? 1 : 0;
        st->max_weight = mx;
        st->max_ratio = per_block ? ratio : mx / st->target;
        if (bal) {
            st->round_done = 1;
        } else {
            // lower bounds shrink with the largest relative influence growth
            st->M = st->M * mu * kDown;
            st->E = st->E * mu * kUp;
            frame_copies(st);
            // the lists stay complete while F <= G sqrt(kListMargin2)
            st->listG = lg;
            st->listF = lf;
            st->lists_ok = lf * lf <= kListMargin2 * (lg * lg) * kDown ? 1 : 0;
            if (sweep_no >= st->max_balance_iter) st->round_done = 1;
        }
    }
}

template <int D>
__global__ __launch_bounds__(1024) void k_balance(RunDev r)
{
    balance_body<D, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
template <int D>
__global__ __launch_bounds__(1024) void k_balance_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    balance_body<D, const RunDev&>(rs[m.x], m.y);
}

// Round end (Alg. 2): the block coordinate sums for the new centers and the
// exact block boxes for beta, the average block diameter of the erosion
// (Sec. 4.2), under the round's final assignment.  One pass block covers
// kPassGroups consecutive 64-point groups and meets all its contributions in
// an LDS table keyed by block, flushed with one set of global atomics per
// distinct block.
//   * sums are kept exactly and incrementally: every point remembers its
//     block at the previous round end, and each group in which a sweep of
//     this round changed a block (marked by the sweep) moves the
//     fixed-point coordinate terms of its changed points from the old
//     block's entry to the new one's;
//   * boxes are rebuilt: a group whose points share one block (recorded by
//     the last sweep) contributes its static box, one lane per group,
//     reduced over runs of equal blocks; the points of mixed groups read
//     their coordinates and touch the table only when they widen it.
// Integer sums and min/max of the order-preserving encoding are exact and
// order-independent, so nothing depends on scheduling.
constexpr int kPassGroups = kBlock;      // one group per thread in the uniform step
// A pass block (16K points) meets far fewer than 128 blocks unless blocks
// hold only a few hundred points, and a full table falls back to the global
// arrays; with 128 slots and two listed groups in flight per wave, 8 waves
// per SIMD fit in LDS and registers.
constexpr int kHashSlots = 128;
constexpr int kMixBatch = 2;             // listed groups a wave has in flight
constexpr int kRoundThreadsMulti = 1024; // threads per block of the many-instance round end

template <int D>
struct RoundTable {
    int key[kHashSlots];
    unsigned long long sum[kHashSlots][2 * D];   // two's complement fixed-point sums
    double box[kHashSlots][2 * D];               // D minima, D maxima
};

// Slot of `key` in the table (inserted if new), or -1 when kProbes probes
// find neither it nor a free slot (the caller then goes to the global
// arrays, which is always valid: the table only batches updates).
constexpr int kProbes = 16;

template <int D>
__device__ inline int table_slot(RoundTable<D>& t, int key)
{
    int slot = (int)(((unsigned)key * 2654435761u) >> 24) & (kHashSlots - 1);
    for (int probe = 0; probe < kProbes; ++probe) {
        const int old = atomicCAS(&t.key[slot], -1, key);
        if (old == -1 || old == key) return slot;
        slot = (slot + 1) & (kHashSlots - 1);
    }
    return -1;
}

// Table slot of every lane's key (lanes with want): one lookup per distinct
// key of the wave, made by a leader lane and broadcast.
template <int D>
__device__ inline int wave_slots(RoundTable<D>& t, int key, bool want)
{
    const int lane = threadIdx.x % kWave;
    unsigned long long pend = __ballot(want);
    int slot = -1;
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int lk = __shfl(key, leader, kWave);
        int ls = 0;
        if (lane == leader) ls = table_slot<D>(t, lk);
        ls = __shfl(ls, leader, kWave);
        const bool mine = want && key == lk;
        if (mine) slot = ls;
        pend &= ~__ballot(mine);
    }
    return slot;
}

template <int CTRL, int ROWS, int D>
__device__ inline void box_step(bool take, unsigned long long* mn, unsigned long long* mx)
{
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const unsigned long long omn = dpp_u64<CTRL, ROWS>(mn[j]);
        const unsigned long long omx = dpp_u64<CTRL, ROWS>(mx[j]);
        mn[j] = take && omn < mn[j] ? omn : mn[j];
        mx[j] = take && omx > mx[j] ? omx : mx[j];
    }
}

// Segmented inclusive min/max over runs of equal `key` across the wave's
// lanes; afterwards the last lane of every run holds the run's box.  Returns
// true on those lanes.  A lane folds in a source lane's value only when the
// source lies in its own run (source index >= run start).
template <int D>
__device__ inline bool run_box(int key, unsigned long long* mn, unsigned long long* mx)
{
    const int lane = threadIdx.x % kWave;
    const int up = __shfl_up(key, 1, kWave);
    const bool head = lane == 0 || key != up;
    const unsigned long long hm = __ballot(head);
    const int start = 63 - __clzll(hm & ((2ULL << lane) - 1ULL));
    const int rl = lane & 15, row = lane >> 4;
    box_step<0x111, 0xf, D>(rl >= 1 && lane - 1 >= start, mn, mx);          // row_shr:1
    box_step<0x112, 0xf, D>(rl >= 2 && lane - 2 >= start, mn, mx);          // row_shr:2
    box_step<0x114, 0xf, D>(rl >= 4 && lane - 4 >= start, mn, mx);          // row_shr:4
    box_step<0x118, 0xf, D>(rl >= 8 && lane - 8 >= start, mn, mx);          // row_shr:8
    box_step<0x142, 0xa, D>((row & 1) && row * 16 - 1 >= start, mn, mx);    // row_bcast:15
    box_step<0x143, 0xc, D>(row >= 2 && 31 >= start, mn, mx);               // row_bcast:31
    return lane == kWave - 1 || ((hm >> (lane + 1)) & 1ULL);
}

// Adds v (or -v) to a slot's sums (or to block c's global sums without a slot).
template <int D>
__device__ inline void add_sums(RoundTable<D>& t, const RunDev& r, int slot, int c,
                                const long long* v, bool negate)
{
    unsigned long long* dst =
        slot >= 0 ? t.sum[slot] : (unsigned long long*)(r.acc + (int64_t)c * kAcc);
#pragma unroll
    for (int j = 0; j < 2 * D; ++j)
        atomicAdd(dst + j, negate ? 0ULL - (unsigned long long)v[j] : (unsigned long long)v[j]);
}

// Widens a slot's box (or block c's global box) by a box, touching an entry
// only when the value improves it (the entries only ever widen, so a stale
// read only lets an update through).
template <int D>
__device__ inline void widen_box(RoundTable<D>& t, const RunDev& r, int slot, int c,
                                 const double* mn, const double* mx)
{
    if (slot >= 0) {
        double* dst = t.box[slot];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (mn[j] < dst[j]) atomicMin(dst + j, mn[j]);
            if (mx[j] > dst[D + j]) atomicMax(dst + D + j, mx[j]);
        }
    } else {
        unsigned long long* dst = r.bb + (int64_t)c * 2 * D;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            atomicMin(dst + j, enc_ord(mn[j]));
            atomicMax(dst + D + j, enc_ord(mx[j]));
        }
    }
}

// NT threads per block: kPassGroups of them take one group each in the
// uniform step; all of them walk the listed groups.
template <int D, bool WEIGHTED, int NT, typename RT>
__device__ __forceinline__ void round_end_body(RT r, const int bid)
{
    const DevState* st = r.st;
    if (st->done || !st->round_done) return;
    __shared__ RoundTable<D> tab;
    __shared__ int s_list[kPassGroups];
    __shared__ int s_n;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    for (int i = tid; i < kHashSlots; i += NT) {
        tab.key[i] = -1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            tab.sum[i][2 * j] = tab.sum[i][2 * j + 1] = 0ULL;
            tab.box[i][j] = INFINITY;
            tab.box[i][D + j] = -INFINITY;
        }
    }
    if (tid == 0) s_n = 0;
    __syncthreads();

    // groups of one block: their static boxes, one lane per group (the
    // first kPassGroups threads)
    const int64_t g0 = (int64_t)bid * kPassGroups;
    const int64_t g = g0 + tid;
    const bool own = tid < kPassGroups;
    // without erosion beta is not needed, and with it no box
    const bool boxes = r.erosion != 0;
    const int f = own && g < r.ngroups ? r.gblk[g] : kPad;
    const bool dirty = own && g < r.ngroups && r.gdirty[g] != 0;
    if (own && boxes) {
        unsigned long long mn[D], mx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            mn[j] = ~0ULL;
            mx[j] = 0ULL;
        }
        if (f >= 0) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                mn[j] = enc_ord(r.gbox[g * 2 * D + j]);
                mx[j] = enc_ord(r.gbox[g * 2 * D + D + j]);
            }
        }
        const bool tail = run_box<D>(f, mn, mx);
        const bool put = tail && f >= 0;
        const int slot = wave_slots<D>(tab, f, put);
        if (put) {
            double dmn[D], dmx[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                dmn[j] = dec_ord(mn[j]);
                dmx[j] = dec_ord(mx[j]);
            }
            widen_box<D>(tab, r, slot, f, dmn, dmx);
        }
    }
    // mixed groups (boxes) and groups with changed points (sums), listed
    if (own) {
        const bool mixed = boxes && f == -1;
        const bool listed = mixed || dirty;
        const unsigned long long b = __ballot(listed);
        int pos = 0;
        if (lane == 0 && b) pos = atomicAdd(&s_n, (int)__popcll(b));
        pos = __shfl(pos, 0, kWave) + (int)__popcll(b & ((1ULL << lane) - 1ULL));
        if (listed) s_list[pos] = tid | (mixed ? 0x100 : 0) | (dirty ? 0x200 : 0);
    }
    __syncthreads();
    const int nl = s_n;
    double lov[D];
#pragma unroll
    for (int j = 0; j < D; ++j) lov[j] = st->lo[j];
    const double sxs = st->sx_scale;
    constexpr int kWaves = NT / kWave;   // every wave of the block walks the list
    for (int m0 = wv * kMixBatch; m0 < nl; m0 += kWaves * kMixBatch) {
        int av[kMixBatch], pv[kMixBatch], ent[kMixBatch];
        double xv[kMixBatch][D];
        // block ids first, then the coordinates the lanes need, so that the
        // loads of the whole batch overlap
#pragma unroll
        for (int u = 0; u < kMixBatch; ++u) {
            // wave-uniform: decisions and addresses on it stay scalar
            ent[u] = __builtin_amdgcn_readfirstlane(m0 + u < nl ? s_list[m0 + u] : 0);
            av[u] = pv[u] = kPad;
            if (m0 + u < nl) {
                const int64_t p = (g0 + (ent[u] & 0xff)) * kWave + lane;
                av[u] = r.A[p];
                pv[u] = (ent[u] & 0x200) ? r.Aprev[p] : av[u];
            }
        }
#pragma unroll
        for (int u = 0; u < kMixBatch; ++u) {
            const bool need = m0 + u < nl && (((ent[u] & 0x100) && av[u] >= 0) || av[u] != pv[u]);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                xv[u][j] = 0.0;
                if (need) {
                    const int64_t p = (g0 + (ent[u] & 0xff)) * kWave + lane;
                    xv[u][j] = r.in_f32 ? (double)r.xs32[j][p] : r.xs64[j][p];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kMixBatch; ++u) {
            if (m0 + u >= nl) break;
            const int64_t gg = g0 + (ent[u] & 0xff);
            const int64_t p = gg * kWave + lane;
            const int a = av[u], ap = pv[u];
            const bool chg = (ent[u] & 0x200) && a != ap;
            // the slot of each lane's block, shared by both steps below
            const int sb = wave_slots<D>(tab, a, a >= 0 && ((ent[u] & 0x100) || chg));
            if (ent[u] & 0x100) {
                // mixed group: every point may widen its block's box
                if (a >= 0) widen_box<D>(tab, r, sb, a, xv[u], xv[u]);
            }
            if (ent[u] & 0x200) {
                // changed points move their terms from the old block to the new
                if (lane == 0) r.gdirty[gg] = 0;
                const unsigned long long cm = __ballot(chg);
                if (cm == 0ULL) continue;
                long long t[2 * D];
                coord_terms<D>(xv[u], lov, WEIGHTED && chg ? r.ws[p] : 1.0, WEIGHTED, sxs, t);
                if (chg) r.Aprev[p] = a;
                if (__popcll(cm) >= 16) {
                    // many changed points (the first round): sum each
                    // (old, new) pair over the wave first
                    unsigned long long pend = cm;
                    while (pend) {
                        const int leader = __builtin_ctzll(pend);
                        const int la = __shfl(ap, leader, kWave);
                        const int lb = __shfl(a, leader, kWave);
                        const bool mine = chg && ap == la && a == lb;
                        const unsigned long long mm = __ballot(mine);
                        long long v[2 * D];
#pragma unroll
                        for (int j = 0; j < 2 * D; ++j) v[j] = wave_sum_dpp(mine ? t[j] : 0);
                        if (lane == leader) {
                            add_sums<D>(tab, r, table_slot<D>(tab, lb), lb, v, false);
                            if (la >= 0) add_sums<D>(tab, r, table_slot<D>(tab, la), la, v, true);
                        }
                        pend &= ~mm;
                    }
                } else {
                    const int sa = wave_slots<D>(tab, ap, chg && ap >= 0);
                    if (chg) {
                        add_sums<D>(tab, r, sb, a, t, false);
                        if (ap >= 0) add_sums<D>(tab, r, sa, ap, t, true);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < kHashSlots; i += NT) {
        const int key = tab.key[i];
        if (key < 0) continue;
        unsigned long long* sums = (unsigned long long*)(r.acc + (int64_t)key * kAcc);
        unsigned long long* box = r.bb + (int64_t)key * 2 * D;
#pragma unroll
        for (int j = 0; j < 2 * D; ++j)
            if (tab.sum[i][j]) atomicAdd(sums + j, tab.sum[i][j]);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (tab.box[i][j] != INFINITY) atomicMin(box + j, enc_ord(tab.box[i][j]));
            if (tab.box[i][D + j] != -INFINITY) atomicMax(box + D + j, enc_ord(tab.box[i][D + j]));
        }
    }
}

template <int D, bool WEIGHTED>
__global__ __launch_bounds__(kBlock, 8) void k_round_end(RunDev r)
{
    round_end_body<D, WEIGHTED, kBlock, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
// (16 waves per block here: an instance may have only a few blocks, whose
// walk over their listed groups must not be long)
template <int D, bool WEIGHTED>
__global__ __launch_bounds__(kRoundThreadsMulti, 2) void k_round_end_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    round_end_body<D, WEIGHTED, kRoundThreadsMulti, const RunDev>(rs[m.x], m.y);
}

// Center movement, convergence, erosion and bound-frame update of one round.
template <int D, typename RT>
__device__ __forceinline__ void move_body(RT r, const int bid)
{
    double* delta = r.red;
    (void)bid;
    DevState* st = r.st;
    if (st->done || !st->round_done) return;
    __shared__ double sh[1024 / kWave];
    const int k = r.k;
    const double sxs = st->sx_scale;
    double dmax = 0.0, dsum = 0.0, cnt = 0.0;
    for (int c = threadIdx.x; c < k; c += 1024) {
        const long long* a = r.acc + (int64_t)c * kAcc;
        const double W = block_weight(r, c);
        double dd = 0.0;
        if (W > 0.0) {
            double cn[D], dv[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                cn[j] = st->lo[j] + (fix_value(a[2 * j], a[2 * j + 1]) / sxs) / W;
                dv[j] = cn[j] - r.C[(int64_t)j * k + c];
            }
            double s = dv[0] * dv[0] + dv[1] * dv[1];
            if (D == 3) s = s + dv[D - 1] * dv[D - 1];
            dd = sqrt(s);
#pragma unroll
            for (int j = 0; j < D; ++j) r.C[(int64_t)j * k + c] = cn[j];
            if (r.erosion) {   // beta, from the block's box
                const unsigned long long* b = r.bb + (int64_t)c * 2 * D;
                double e[D];
#pragma unroll
                for (int j = 0; j < D; ++j) e[j] = dec_ord(b[D + j]) - dec_ord(b[j]);
                double q = e[0] * e[0] + e[1] * e[1];
                if (D == 3) q = q + e[D - 1] * e[D - 1];
                dsum += sqrt(q);
            }
            cnt += 1.0;
        }
        delta[c] = dd;
        dmax = fmax(dmax, dd);
    }
    dmax = block_reduce_1024(dmax, sh, OpMax());
    dsum = block_reduce_1024(dsum, sh, OpAdd());
    cnt = block_reduce_1024(cnt, sh, OpAdd());
    const bool conv = dmax < st->delta_threshold;
    const double beta = r.erosion ? dsum / cnt : 0.0;
    double mu = 1.0, emax = 0.0;
    if (!conv) {
        double m = INFINITY, e = 0.0;
        for (int c = threadIdx.x; c < k; c += 1024) {
            const double dl = delta[c];
            const double io = r.I[c];
            double in = io;
            if (dl != 0.0 && r.erosion) {
                double t = -dl / beta;
                if (t > 0.0) t = 0.0;
                const double alpha = 2.0 / (1.0 + exp(t)) - 1.0;
                in = exp((1.0 - alpha) * log(io));
            }
            r.I[c] = in;
            const double dacc = (r.clus[c].x + dl) * kUp;
            r.clus[c] = make_double2(dacc, 1.0 / in);
            r.clus32[c] = make_float2(f32_up(dacc), f32_up(1.0 / in));
            r.clusdn[c] = f32_down(dacc);
            m = fmin(m, io / in);
            e = fmax(e, dl / in);
            // after the balance step of the same interval
            r.cdec[c] = make_double2(r.cdec[c].x * (io / in), dl / in);
        }
        mu = block_reduce_1024(m, sh, OpMin());
        emax = block_reduce_1024(e, sh, OpMax());
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->max_delta = dmax;
        st->beta = beta;
        st->nonempty = (int)cnt;
        st->rounds += 1;
        if (conv) {
            st->converged = 1;
            st->done = 1;
        } else {
            st->M = st->M * mu * kDown;
            st->E = (st->E * mu + emax) * kUp;
            frame_copies(st);
            st->imu = st->imu * mu;
            st->ie = emax;
        }
        if (st->rounds >= st->max_iter) st->done = 1;
        st->round_done = 0;
        st->sweep_in_round = 0;
        st->lists_ok = 0;   // the centers moved: the next sweep rebuilds the lists
    }
    for (int i = threadIdx.x; i < k * 2 * D; i += 1024) r.bb[i] = (i % (2 * D)) < D ? ~0ULL : 0ULL;
}

template <int D>
__global__ __launch_bounds__(1024) void k_move(RunDev r)
{
    move_body<D, const RunDev>(r, blockIdx.x);
}

// Many instances in one launch: block b works on instance map[b].x as its
// block map[b].y.
template <int D>
__global__ __launch_bounds__(1024) void k_move_multi(const RunDev* rs, const int2* map)
{
    const int2 m = map[blockIdx.x];
    move_body<D, const RunDev&>(rs[m.x], m.y);
}

// Fresh run state: influence 1, no assignment, empty sums, open bounds.
__global__ __launch_bounds__(kBlock) void k_init_points(RunDev r)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= r.npad) return;
    r.A[i] = r.perm[i] >= 0 ? -1 : kPad;
    r.Aprev[i] = r.A[i];
    r.bnd[i] = make_float2(INFINITY, 0.0f);
    if (i < r.ngroups) r.gdirty[i] = 0;
    if (i < r.ntiles) {
        TileBound f;
        f.M = 1.0;
        f.E = 0.0;
        f.Mf = 1.0f;
        f.Ef = 0.0f;
        f.Edn = 0.0f;
        f.invMdn = f32_down(1.0 - 0x1p-21);
        f.lam = INFINITY;
        f.pad = 0.0f;
        r.tbnd[i] = f;
    }
}

// Non-uniform target sizes (the footnote to the objective at the start of
// Sec. 4).  Prefix sums of the caller's relative sizes are taken in index
// order by one thread over chunks staged in LDS (the order fixes the
// rounding); then every block gets its target weight W*t/tsum and its limit,
// (1+eps)*ceil(n*t/tsum) for unit weights or (1+eps)*target for node
// weights, and the largest limit goes to the state.  A size that is not
// finite and positive, or a total that overflows, sets bad_data bit 4.
constexpr int kPrepChunk = 4096;

__global__ __launch_bounds__(1024) void k_target_prep(RunDev r, double eps)
{
    __shared__ double buf[kPrepChunk];
    __shared__ double sh[1024 / kWave];
    __shared__ double total;
    __shared__ int bad;
    const int k = r.k;
    double run = 0.0;
    int b = 0;
    for (int base = 0; base < k; base += kPrepChunk) {
        const int m = min(kPrepChunk, k - base);
        for (int i = threadIdx.x; i < m; i += 1024) buf[i] = r.tsz[base + i];
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 0; i < m; ++i) {
                const double t = buf[i];
                r.tpre[base + i] = run;
                if (!(t > 0.0) || !isfinite(t)) b = 1;
                run += t;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        r.tpre[k] = run;
        if (!isfinite(run)) b = 1;
        total = run;
        bad = b;
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) atomicOr(&r.st->bad_data, 4);
        return;
    }
    const double W = r.st->total_weight;
    const double tsum = total;
    double lm = 0.0;
    for (int c = threadIdx.x; c < k; c += 1024) {
        const double t = r.tsz[c];
        const double T = (W * t) / tsum;
        const double L = r.weighted ? (1.0 + eps) * T
                                    : (1.0 + eps) * ceil(((double)r.n * t) / tsum);
        r.tT[c] = T;
        r.tL[c] = L;
        lm = fmax(lm, L);
    }
    lm = block_reduce_1024(lm, sh, OpMax());
    if (threadIdx.x == 0) r.st->lmax = lm;
}

__global__ __launch_bounds__(kBlock) void k_init_clusters(RunDev r, const double* cinit,
                                                          const double* iinit, int max_iter,
                                                          int max_bal, double eps, double dthr)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const int D = r.d;
    if (c < kCntSlots * kCntWords) r.cnt[c] = 0;
    if (c < r.k) {
        if (cinit)
            for (int j = 0; j < D; ++j) r.C[(int64_t)j * r.k + c] = cinit[(int64_t)c * D + j];
        const double in = iinit ? iinit[c] : 1.0;
        r.I[c] = in;
        r.clus[c] = make_double2(0.0, 1.0 / in);
        r.clus32[c] = make_float2(0.0f, f32_up(1.0 / in));
        r.clusdn[c] = 0.0f;
        r.cdec[c] = make_double2(1.0, 0.0);
        for (int a = 0; a < kAcc; ++a) r.acc[(int64_t)c * kAcc + a] = 0;
        for (int j = 0; j < 2 * D; ++j) r.bb[(int64_t)c * 2 * D + j] = j < D ? ~0ULL : 0ULL;
    }
    if (c == 0) {
        DevState* st = r.st;
        st->done = 0;
        st->round_done = 0;
        st->balanced = 0;
        st->converged = 0;
        st->rounds = 0;
        st->sweep_in_round = 0;
        st->sweeps = 0;
        st->max_iter = max_iter;
        st->max_balance_iter = max_bal;
        st->M = 1.0;
        st->E = 0.0;
        frame_copies(st);
        st->lists_ok = 0;
        st->listG = 1.0;
        st->listF = 1.0;
        st->imu = 1.0;
        st->ie = 0.0;
        const double W = st->total_weight;
        if (!r.tsz) {   // with target sizes, the prep left the largest limit here
            if (r.weighted) {
                st->lmax = (1.0 + eps) * (W / (double)r.k);
            } else {
                const int64_t ck = (r.n + r.k - 1) / r.k;
                st->lmax = (1.0 + eps) * (double)ck;
            }
        }
        st->target = W / (double)r.k;
        st->delta_threshold = dthr < 0.0 ? 1e-5 * st->ext : dthr;
    }
}

// Caller-given centers/influence of one step of bkm_assign_sweeps, with the
// bound relaxation the change implies (movement delta, influence ratios).
template <int D>
__global__ __launch_bounds__(1024) void k_set_step(RunDev r, const double* crm,
                                                   const double* infl, int first)
{
    DevState* st = r.st;
    __shared__ double sh[1024 / kWave];
    const int k = r.k;
    double m = INFINITY, e = 0.0;
    for (int c = threadIdx.x; c < k; c += 1024) {
        double dv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double v = crm[(int64_t)c * D + j];
            dv[j] = v - r.C[(int64_t)j * k + c];
            r.C[(int64_t)j * k + c] = v;
        }
        double s = dv[0] * dv[0] + dv[1] * dv[1];
        if (D == 3) s = s + dv[D - 1] * dv[D - 1];
        const double dl = first ? 0.0 : sqrt(s);
        const double io = r.I[c];
        const double in = infl[c];
        r.I[c] = in;
        const double dacc = first ? 0.0 : (r.clus[c].x + dl) * kUp;
        r.clus[c] = make_double2(dacc, 1.0 / in);
        r.clus32[c] = make_float2(f32_up(dacc), f32_up(1.0 / in));
        r.clusdn[c] = f32_down(dacc);
        r.cdec[c] = make_double2(io / in, dl / in);
        m = fmin(m, io / in);
        e = fmax(e, dl / in);
    }
    m = block_reduce_1024(m, sh, OpMin());
    e = block_reduce_1024(e, sh, OpMax());
    __syncthreads();
    if (threadIdx.x == 0) {
        if (first) {
            st->M = 1.0;
            st->E = 0.0;
        } else {
            st->M = st->M * m * kDown;
            st->E = (st->E * m + e) * kUp;
        }
        frame_copies(st);
        st->imu = m;
        st->ie = e;
        st->done = 0;
        st->round_done = 0;
        st->lists_ok = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter_back(RunDev r, int32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < r.npad) {
        const int32_t src = r.perm[i];
        if (src >= 0) out[src] = r.A[i];
    }
}

__global__ __launch_bounds__(kBlock) void k_cluster_out(RunDev r, double* cout, double* iout,
                                                        double* bwout)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= r.k) return;
    if (cout)
        for (int j = 0; j < r.d; ++j) cout[(int64_t)c * r.d + j] = r.C[(int64_t)j * r.k + c];
    if (iout) iout[c] = r.I[c];
    if (bwout) bwout[c] = block_weight(r, c);
}

// ---------------------------------------------------------------- statistics
// partition_stats works on the caller's points in input order.
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_stats_sums(RunDev r, const int32_t* asg)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x % kWave;
    const bool valid = i < r.n;
    int a = valid ? asg[i] : 0;
    if (valid && (a < 0 || a >= r.k)) {
        atomicOr(&r.st->bad_data, 2);
        a = 0;
    }
    const DevState* st = r.st;
    long long th[D], tl[D], wh = 1, wl = 0;
    const double w = (valid && r.in_w) ? r.in_w[i] : 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double v = valid ? (double)((const T*)r.in_x[j])[i] - st->lo[j] : 0.0;
        if (r.in_w) v = w * v;
        fix_split(v * st->sx_scale, th[j], tl[j]);
    }
    if (r.in_w) fix_split(w * st->w_scale, wh, wl);
    unsigned long long pend = __ballot(valid);
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int key = __shfl(a, leader, kWave);
        const bool mine = valid && a == key;
        const unsigned long long mm = __ballot(mine);
        long long v[kAcc];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            v[2 * j] = wave_sum_ll(mine ? th[j] : 0);
            v[2 * j + 1] = wave_sum_ll(mine ? tl[j] : 0);
        }
        v[6] = r.in_w ? wave_sum_ll(mine ? wh : 0) : (long long)__popcll(mm);
        v[7] = r.in_w ? wave_sum_ll(mine ? wl : 0) : 0;
        if (lane == leader) {
            unsigned long long* dst = (unsigned long long*)(r.acc + (int64_t)key * kAcc);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                atomicAdd(dst + 2 * j, (unsigned long long)v[2 * j]);
                atomicAdd(dst + 2 * j + 1, (unsigned long long)v[2 * j + 1]);
            }
            atomicAdd(dst + 6, (unsigned long long)v[6]);
            atomicAdd(dst + 7, (unsigned long long)v[7]);
        }
        pend &= ~mm;
    }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_stats_centers(RunDev r, double* bwout,
                                                          double* cout)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= r.k) return;
    const long long* a = r.acc + (int64_t)c * kAcc;
    const double W = block_weight(r, c);
    if (bwout) bwout[c] = W;
    for (int j = 0; j < D; ++j) {
        const double v = W > 0.0 ? r.st->lo[j] + (fix_value(a[2 * j], a[2 * j + 1]) / r.st->sx_scale) / W
                                 : NAN;
        r.C[(int64_t)j * r.k + c] = v;
        if (cout) cout[(int64_t)c * D + j] = v;
    }
}

// Per-block partial objective sums in a fixed order (deterministic).
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_stats_objective(RunDev r, const int32_t* asg)
{
    __shared__ double sh[kBlock / kWave];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < r.n; i += stride) {
        int a = asg[i];
        if (a < 0 || a >= r.k) continue;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double dv = (double)((const T*)r.in_x[j])[i] - r.C[(int64_t)j * r.k + a];
            s = s + dv * dv;
        }
        acc += (r.in_w ? r.in_w[i] : 1.0) * s;
    }
    acc = wave_sum_d(acc);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) t += sh[w];
        r.red[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_stats_final(RunDev r, int nparts, double eps,
                                                        double* out6)
{
    __shared__ double sh[kBlock / kWave];
    double mx = 0.0, empty = 0.0, over = 0.0;
    const DevState* st = r.st;
    const double W = st->total_weight;
    double lmax;
    if (r.weighted) {
        lmax = (1.0 + eps) * (W / (double)r.k);
    } else {
        const int64_t ck = (r.n + r.k - 1) / r.k;
        lmax = (1.0 + eps) * (double)ck;
    }
    // with target sizes mx is the largest weight / target, and every block
    // has its own limit
    for (int c = threadIdx.x; c < r.k; c += kBlock) {
        const double b = block_weight(r, c);
        if (r.tsz) {
            mx = fmax(mx, b / r.tT[c]);
            if (b > r.tL[c]) over += 1.0;
        } else {
            mx = fmax(mx, b);
            if (b > lmax) over += 1.0;
        }
        if (b == 0.0) empty += 1.0;
    }
    mx = wave_max_d(mx);
    empty = wave_sum_d(empty);
    over = wave_sum_d(over);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int w = 1; w < kBlock / kWave; ++w) m = fmax(m, sh[w]);
        out6[0] = r.tsz ? m - 1.0 : m / (W / (double)r.k) - 1.0;
        double obj = 0.0;
        for (int b = 0; b < nparts; ++b) obj += r.red[b];
        out6[1] = obj;
        out6[2] = r.tsz ? st->lmax : lmax;
    }
    __syncthreads();
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = empty;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) e += sh[w];
        out6[3] = e;
    }
    __syncthreads();
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = over;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) e += sh[w];
        out6[4] = e;
        out6[5] = (double)st->bad_data;
    }
}

inline unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_target_prep(const RunDev& r, double eps, hipStream_t s)
{
    k_target_prep<<<1, 1024, 0, s>>>(r, eps);
    return hipGetLastError();
}

hipError_t launch_init_run(const RunDev& r, const double* cinit, const double* iinit, int max_iter,
                           int max_balance_iter, double eps, double dthr, hipStream_t s)
{
    k_init_points<<<nblocks(r.npad, kBlock), kBlock, 0, s>>>(r);
    k_init_clusters<<<nblocks(std::max(r.k, kCntSlots * kCntWords), kBlock), kBlock, 0, s>>>(
        r, cinit, iinit, max_iter, max_balance_iter, eps, dthr);
    return hipGetLastError();
}

hipError_t launch_balance(const RunDev& r, hipStream_t s)
{
    if (r.d == 2)
        k_balance<2><<<1, 1024, 0, s>>>(r);
    else
        k_balance<3><<<1, 1024, 0, s>>>(r);
    return hipGetLastError();
}

hipError_t launch_block_boxes(const RunDev& r, hipStream_t s)
{
    const unsigned g = (unsigned)((r.ngroups + kPassGroups - 1) / kPassGroups);
    if (r.d == 2) {
        if (r.weighted) k_round_end<2, true><<<g, kBlock, 0, s>>>(r);
        else k_round_end<2, false><<<g, kBlock, 0, s>>>(r);
    } else {
        if (r.weighted) k_round_end<3, true><<<g, kBlock, 0, s>>>(r);
        else k_round_end<3, false><<<g, kBlock, 0, s>>>(r);
    }
    return hipGetLastError();
}

// Debug check of the Hamerly invariants (Sec. 4.3) on sampled points, all in
// exact FP64 against every center: the stored upper bound plus the movement
// of the point's center is at least its distance to that center; the lower
// bound in its affine frame (M * stored - E) is at most the effective
// distance to every other center; and, right after a sweep, the point's
// block is an argmin of the effective distance (within the 1e-12 tie gap).
// Relative slack 1e-12 on each side.  Violations are counted, not trapped.
template <int D>
__global__ __launch_bounds__(kBlock) void k_check_bounds(RunDev r, int after_sweep)
{
    const DevState* st = r.st;
    if (after_sweep ? round_over(st) : st->done != 0) return;
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * r.debug_stride;
    bool checked = false, bad = false;
    if (i < r.npad) {
        const int a = r.A[i];
        if (a != kPad) {
            checked = true;
            if (a < 0 || a >= r.k) {
                bad = true;
            } else {
                double x[D];
#pragma unroll
                for (int j = 0; j < D; ++j)
                    x[j] = r.in_f32 ? (double)r.xs32[j][i] : r.xs64[j][i];
                const int k = r.k;
                double own = 0.0, own_sq = 0.0, other = INFINITY, best = INFINITY;
                for (int c = 0; c < k; ++c) {
                    const double dx = x[0] - r.C[c];
                    const double dy = x[1] - r.C[(int64_t)k + c];
                    double sq = dx * dx + dy * dy;
                    if (D == 3) {
                        const double dz = x[2] - r.C[(int64_t)(D - 1) * k + c];
                        sq = sq + dz * dz;
                    }
                    const double e = sqrt(sq) / r.I[c];
                    best = fmin(best, e);
                    if (c == a) {
                        own = e;
                        own_sq = sq;
                    } else {
                        other = fmin(other, e);
                    }
                }
                const float2 b = r.bnd[i];
                const double ub = (double)b.x + r.clus[a].x;
                // the tile's frame; after a center move, with the move's
                // relaxation over all centers (the next sweep's tile
                // candidates apply their own)
                const TileBound& f = r.tbnd[i / r.T];
                double lb = f.M * fmin((double)b.y, (double)f.lam) - f.E;
                if (!after_sweep) lb = st->imu * lb - st->ie;
                if (ub < sqrt(own_sq) * (1.0 - 1e-12)) bad = true;
                if (lb > other * (1.0 + 1e-12)) bad = true;
                if (after_sweep && own > best * (1.0 + 1e-12)) bad = true;
            }
        }
    }
    const unsigned long long nc = __popcll(wave_ballot(checked));
    const unsigned long long nb = __popcll(wave_ballot(bad));
    if (threadIdx.x % kWave == 0 && nc) {
        unsigned long long* slot = r.cnt + (int64_t)(blockIdx.x % kCntSlots) * kCntWords;
        atomicAdd(slot + kCntDebugChecked, nc);
        if (nb) atomicAdd(slot + kCntDebugViolated, nb);
    }
}

hipError_t launch_check_bounds(const RunDev& r, int after_sweep, hipStream_t s)
{
    if (r.debug_stride <= 0) return hipSuccess;
    const int64_t m = (r.npad + r.debug_stride - 1) / r.debug_stride;
    const unsigned g = nblocks(m, kBlock);
    if (r.d == 2)
        k_check_bounds<2><<<g, kBlock, 0, s>>>(r, after_sweep);
    else
        k_check_bounds<3><<<g, kBlock, 0, s>>>(r, after_sweep);
    return hipGetLastError();
}

hipError_t launch_move(const RunDev& r, hipStream_t s)
{
    if (r.d == 2)
        k_move<2><<<1, 1024, 0, s>>>(r);
    else
        k_move<3><<<1, 1024, 0, s>>>(r);
    return hipGetLastError();
}

hipError_t launch_set_step(const RunDev& r, const double* crm, const double* infl, int first,
                           hipStream_t s)
{
    if (r.d == 2)
        k_set_step<2><<<1, 1024, 0, s>>>(r, crm, infl, first);
    else
        k_set_step<3><<<1, 1024, 0, s>>>(r, crm, infl, first);
    return hipGetLastError();
}

hipError_t launch_finish(const RunDev& r, int32_t* asg, double* cout, double* iout,
                         double* bwout, hipStream_t s)
{
    if (asg) k_scatter_back<<<nblocks(r.npad, kBlock), kBlock, 0, s>>>(r, asg);
    k_cluster_out<<<nblocks(r.k, kBlock), kBlock, 0, s>>>(r, cout, iout, bwout);
    return hipGetLastError();
}

hipError_t launch_stats(const RunDev& r, const int32_t* asg, double eps, double* bwout,
                        double* cout, double* out6, hipStream_t s)
{
    const unsigned g = nblocks(r.n, kBlock);
    const int nparts = (int)std::min<int64_t>(1024, g);
    if (r.d == 2) {
        if (r.in_f32) k_stats_sums<float, 2><<<g, kBlock, 0, s>>>(r, asg);
        else k_stats_sums<double, 2><<<g, kBlock, 0, s>>>(r, asg);
        k_stats_centers<2><<<nblocks(r.k, kBlock), kBlock, 0, s>>>(r, bwout, cout);
        if (r.in_f32) k_stats_objective<float, 2><<<nparts, kBlock, 0, s>>>(r, asg);
        else k_stats_objective<double, 2><<<nparts, kBlock, 0, s>>>(r, asg);
    } else {
        if (r.in_f32) k_stats_sums<float, 3><<<g, kBlock, 0, s>>>(r, asg);
        else k_stats_sums<double, 3><<<g, kBlock, 0, s>>>(r, asg);
        k_stats_centers<3><<<nblocks(r.k, kBlock), kBlock, 0, s>>>(r, bwout, cout);
        if (r.in_f32) k_stats_objective<float, 3><<<nparts, kBlock, 0, s>>>(r, asg);
        else k_stats_objective<double, 3><<<nparts, kBlock, 0, s>>>(r, asg);
    }
    k_stats_final<<<1, kBlock, 0, s>>>(r, nparts, eps, out6);
    return hipGetLastError();
}

template <int D>
hipError_t update_multi_d(const MultiSet& m, hipStream_t s)
{
    k_balance_multi<D><<<m.ninst, 1024, 0, s>>>(m.rs, m.map_inst);
    if (m.nb_pass) {
        if (m.weighted) k_round_end_multi<D, true><<<m.nb_pass, kRoundThreadsMulti, 0, s>>>(m.rs, m.map_pass);
        else k_round_end_multi<D, false><<<m.nb_pass, kRoundThreadsMulti, 0, s>>>(m.rs, m.map_pass);
    }
    k_move_multi<D><<<m.ninst, 1024, 0, s>>>(m.rs, m.map_inst);
    return hipGetLastError();
}

hipError_t launch_update_multi(const MultiSet& m, hipStream_t s)
{
    static_assert(kPassGroups == kPassGroupsHost, "round-end pass geometry");
    return m.d == 2 ? update_multi_d<2>(m, s) : update_multi_d<3>(m, s);
}

}  // namespace bkm
