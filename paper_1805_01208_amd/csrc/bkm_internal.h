// Internal declarations of libbkm: device state, the device-memory layout of one
// run, launch wrappers and wave-level helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

#include "bkm.h"

namespace bkm {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per block of the point kernels
constexpr int kTileCap = 128;        // candidate records kept per tile
constexpr int kHyper = 16;           // super-tiles per hyper-tile of the candidate hierarchy
// Squared margin of the candidate filters (Sec. 4.4 filter, widened): a
// list keeps every center whose smallest effective distance to the box is
// within sqrt(kListMargin2) of the second-smallest largest one, so it stays
// complete while every center's 1/influence moves by a ratio in [G, F]
// with F <= G sqrt(kListMargin2); the lists are then kept.
constexpr double kListMargin2 = 1.3125;
constexpr int kFixShift = 30;        // fixed-point sums: term = hi * 2^30 + lo
constexpr long long kFixLoMask = (1LL << kFixShift) - 1;
constexpr int kPad = -2;             // block id of a padding point (never evaluated)
constexpr int kMaxJumps = 8192;      // jumps between Hilbert-consecutive points realigned to tiles
constexpr int kGapBins = 128;        // log2 histogram of gaps between consecutive points
constexpr int kCntSlots = 64;        // sweep counters spread over this many cache lines
constexpr int kCntWords = 16;        // counters per slot (one 128-byte line)
constexpr int kSortIpt = 8;          // radix sort: items per thread per pass
constexpr int kSortChunk = kBlock * kSortIpt;   // items per block per pass

// Control and scalar state of one run, resident in device memory.  Kernels
// of a round read it to decide whether they still have work (a finished
// AssignAndBalance call or a finished run turns later launches into no-ops),
// so the host only synchronises once per round.
struct alignas(16) DevState {
    int32_t done;             // run finished (converged or out of rounds)
    int32_t round_done;       // current AssignAndBalance call finished (right after done:
                              // both are read as one 8-byte word)
    int32_t balanced;         // result of the last balance test
    int32_t converged;
    int32_t rounds;           // AssignAndBalance calls completed
    int32_t sweep_in_round;   // sweeps made in the current call
    int32_t sweeps;           // sweeps made in total
    int32_t max_iter;
    int32_t max_balance_iter;
    int32_t bad_data;         // a non-finite coordinate or a bad weight was seen
    int32_t nonempty;         // non-empty blocks seen by the last center update
    int32_t njumps;           // jumps found (before the kMaxJumps / capacity cap)
    int64_t npad;             // padded point count of the tiled layout
    // Hamerly lower bounds are stored in a lazy frame: the bound at the current
    // time is M * stored - E (both conservatively rounded).
    double M, E;
    double lmax, target, delta_threshold;
    double lo[3], hi[3];      // global bounding box
    double ext;               // largest extent
    double key_scale;         // 2^m / ext for the Hilbert cells
    double sx_scale;          // power of two: coordinate term = rint(w*(x-lo)*sx_scale)
    double w_scale;           // power of two: weight term = rint(w*w_scale) (1 for unit weights)
    double wmax;
    double beta, max_delta, max_weight, total_weight;
    double max_ratio;         // largest weight / target over the blocks at the last balance test
    // Candidate lists are built with a margin and kept while the influences
    // move within it: listG and listF bound (1/I now) / (1/I at the last
    // build) over all centers from below and above; the balance step keeps
    // them (they mean something only while lists_ok is set).
    double listG, listF;
    double jump_thr2;         // squared gap above which consecutive points start a new tile
    // (r, s) over all centers for the last interval between sweeps (the
    // debug check after a center move relaxes the tile bounds with them)
    double imu, ie;
    // the sweep's copies of the frame, refreshed wherever M or E change
    double invM;              // 1 / M
    float Mf, Ef;             // M rounded down and E rounded up to FP32
    float Edn, invMdn;        // E rounded down; 1/M times (1 - 2^-21), rounded down
    int32_t lists_ok;         // 1: the next sweep keeps the candidate lists of the last build;
                              // 0: they are rebuilt
};

// The run or the current AssignAndBalance call is over: one 8-byte load of
// the two adjacent flags.
__device__ inline bool round_over(const DevState* st)
{
    const int2 f = *reinterpret_cast<const int2*>(&st->done);
    return (f.x | f.y) != 0;
}

// Sweep counters, summed over the kCntSlots slots by the host.
enum {
    kCntEvaluated = 0, kCntSkipped, kCntRechecked, kCntChanged, kCntCandEvals, kCntOverflow,
    kCntInvalid,      // decisions that produced no valid block (an internal error)
    kCntDebugChecked, // debug checks: points checked
    kCntDebugViolated, // debug checks: points whose bounds or block failed the check
    kCntListBuilds    // sweeps that built the candidate lists (the others kept them)
};

// Candidates of one tile for the current sweep, written by k_tilecand.
struct TileHead {
    int32_t n;                // records in use
    int32_t overflow;         // 1: more than kTileCap candidates; sweep the super-tile list
    float step[3];            // FP32 value of one unit of the tile's fixed-point offsets, per axis
    float slack32;            // FP32 screen slack: tau(1 + 16u) + 2^-46, rounded up
    double tau;               // bound on |FP32 effective distance - exact| over the candidates
    double dmax;              // bound on |FP32 distance - exact| over the candidates
    double lb_out;            // lower bound on the effective distance of every center left out
    float ubadd32;            // dmax + 2^-46 (1 + 7u), rounded up: the upper bound's additive term
    float lbout32;            // lb_out rounded down
    double lb_build;          // lb_out at the build
};

// Lower-bound frame of a tile (Sec. 4.3 bounds, relaxed per tile).  The
// points of a tile store their Hamerly lower bound lb as s = (lb + E) / M.
// Between two sweeps every center's effective distances change by at least
// a ratio r_c (influence) and a shift s_c (movement); the second-best
// center of a point of the tile is then one of the tile's candidates (their
// ratios and shifts bound the change) or a center left out of its list
// (whose distance is at least the list's fresh lb_out), so the bound of the
// next sweep is min(m lb - e, lb_out) with m, e the smallest ratio and
// largest shift over the tile's candidates: the frame takes M <- m M,
// E <- m E + e, and the sweep lowers a stored s above lam = (lb_out + E) / M
// to lam.  FP32 copies are rounded so that every bound stays valid.
struct TileBound {
    double M, E;
    float Mf, Ef;             // M rounded down, E rounded up
    float Edn, invMdn;        // E rounded down; 1/M times (1 - 2^-21), rounded down
    float lam;                // lam rounded down
    float pad;
};

// Static frame of a tile, fixed by its box at the layout: the anchor X (box
// center) of the packed offsets, the norm of the box half-extents, and the
// FP32 value of one unit of the offsets per axis.
struct TileFrame {
    double X[3];
    double hnorm;
    float step[3];
    float pad;
};

// One candidate center of a tile: FP32 offset of the center from the tile
// anchor and squared FP32 inverse influence, for the FP32 screen, and a lower
// bound (key) on the value the screen (or the FP64 sweep) can compute for
// this center at any point of the tile.  A tile's records are sorted by that
// key.  dlt and key0 keep what the build knew: the center's term of the FP32
// error bound before 1/influence (rounded up) and the key, from which a
// sweep that keeps the lists refreshes w2, key and the tile's bounds.
struct alignas(32) CandRec {
    float qx, qy, qz, w2;
    int32_t id;
    float key;
    float dlt, key0;
};

// Everything a run keeps on the device.  Point arrays are in Hilbert (sorted)
// order and padded to whole tiles.
struct RunDev {
    int64_t n, npad, npad_cap;  // points, padded layout size, its capacity
    int d, k, in_f32, weighted;
    int maxjumps;
    int T, ppt, ntiles, super_tiles, nsuper, nhyper, ngroups;
    int precision, use_bounds;
    int erosion;              // 1: erode the influence after every non-converged movement
    int debug_stride;         // > 0: check every debug_stride-th layout slot after each
                              // sweep and each move (bounds, block) against brute force
    double recheck_gap;

    const void* in_x[3];      // caller's coordinates (input order)
    const double* in_w;       // caller's weights or null
    const double* tsz;        // caller's relative target sizes [k], or null (equal blocks)

    double* xs64[3];          // sorted master coordinates (FP64 input)
    float* xs32[3];           // sorted master coordinates (FP32 input)
    void* ofs;                // packed fixed-point offsets from the tile anchor, one word
                              // per point (FP32 sweep): 2D 32 bits, 3D 64 bits
    double* ws;               // sorted weights or null
    int32_t* sperm;           // Hilbert order -> input index (n entries, no padding)
    int32_t* perm;            // padded layout position -> input index, -1 for padding
    double* tx64[3];          // coordinates in Hilbert order before padding (FP64 input)
    float* tx32[3];           // same for FP32 input
    unsigned int* ghist;      // [kGapBins]
    int32_t* jumps;           // [maxjumps] first point after each jump, sorted by the plan
    int64_t* jshift;          // [maxjumps] layout shift of the points from jumps[j] on
    int32_t* A;               // current block of each sorted point (-1: none yet)
    float2* bnd;              // stored bounds of each point: x upper (distance frame),
                              // y lower (lazy frame), one 8-byte record
    double* tbox;             // [ntiles][2d] lo..., hi...
    TileFrame* tframe;        // [ntiles]
    TileBound* tbnd;          // [ntiles] lower-bound frames
    double2* cdec;            // [k] (r_c, s_c): smallest ratio and largest shift of the center's
                              // effective distances since the last sweep
    double* gbox;             // [ngroups][2d] boxes of 64-point groups
    double* hbox;             // [nhyper][2d] boxes of hyper-tiles (kHyper super-tiles)
    int32_t* hlist;           // [nhyper][k] candidate centers of each hyper-tile
    int32_t* hcount;          // [nhyper]
    double* sbox;             // [nsuper][2d]
    int32_t* slist;           // [nsuper][k] candidate centers of each super-tile
    int32_t* scount;          // [nsuper]
    TileHead* thead;          // [ntiles]
    CandRec* tcand;           // [ntiles][kTileCap]
    double* C;                // [d][k] centers (SoA)
    double* I;                // [k] influence
    double* tT;               // [k] target weight of each block (with target sizes)
    double* tL;               // [k] weight limit of each block (with target sizes)
    double* tpre;             // [k+1] prefix sums of the target sizes in index order; [k] = total
    double2* clus;            // [k] (accumulated movement, 1/influence)
    double* ivb;              // [k] 1/influence at the last candidate-list build
    float2* clus32;           // [k] FP32 copies for the Hamerly test: movement and
                              // 1/influence, both rounded up
    float* clusdn;            // [k] movement rounded down to FP32 (bound stores)
    int32_t* Aprev;           // [npad] block of each point at the previous round end
    int32_t* gdirty;          // [ngroups] 1 if a point of the group changed block in this round
    int32_t* gblk;            // [ngroups] block of every point of the group after the last
                              // sweep; -1 if they may differ (always when a point of the
                              // group changed block in it); kPad if all padding
    long long* acc;           // [k][kAcc] fixed-point block sums
    unsigned long long* bb;   // [k][2d] encoded block boxes (min..., max...)
    DevState* st;
    unsigned long long* cnt;  // [kCntSlots][kCntWords]
    // bootstrap scratch
    uint64_t* keys;
    uint64_t* keys2;
    int32_t* vals2;
    uint32_t* hist;
    uint32_t* part;
    double* red;              // per-block partial reductions
};

// Number of fixed-point accumulators per block: coordinate hi/lo per axis and
// weight hi/lo (count in the hi word for unit weights).  The weights follow
// every sweep incrementally; the coordinate sums are rebuilt at the end of
// each AssignAndBalance call.
constexpr int kAcc = 8;
constexpr int kAccW = 6;

// Fixed-point coordinate terms of one point: hi/lo words of
// rint(w * (x_j - lo_j) * sx_scale) per axis (w = 1 for unit weights).
template <int D>
__device__ inline void coord_terms(const double* x, const double* lo, double w, bool weighted,
                                   double sxs, long long* t)
{
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double v = x[j] - lo[j];
        if (weighted) v = w * v;
        long long h, l;
        const long long q = __double2ll_rn(v * sxs);
        h = q >> kFixShift;
        l = q & kFixLoMask;
        t[2 * j] = h;
        t[2 * j + 1] = l;
    }
}

// Fixed-point point offsets of the FP32 screen: per tile and axis, the
// offset from the tile anchor X (box center) in units of h/FixMax, h the box
// half-extent on that axis, rounded to nearest; one packed word per point:
// 2D two 16-bit fields in 32 bits, 3D three 21-bit fields in 64 bits.
template <int D> struct FixPack;
template <> struct FixPack<2> {
    using word = uint32_t;
    static constexpr int kBits = 16;
    static constexpr double kMax = 32767.0;
};
template <> struct FixPack<3> {
    using word = unsigned long long;
    static constexpr int kBits = 21;
    static constexpr double kMax = 1048575.0;
};

// Field value of offset v on an axis of half-extent h.
template <int D>
__device__ inline long long fix_offset(double v, double h)
{
    constexpr double m = FixPack<D>::kMax;
    if (!(h > 0.0)) return 0;
    double q = rint(v / h * m);
    q = fmin(fmax(q, -m), m);
    return (long long)q;
}

template <int D>
__device__ inline typename FixPack<D>::word fix_pack(const long long* q)
{
    using W = typename FixPack<D>::word;
    constexpr int b = FixPack<D>::kBits;
    constexpr W mask = (W(1) << b) - 1;
    W w = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) w |= ((W)q[j] & mask) << (b * j);
    return w;
}

// Field j of a packed word, sign-extended, as FP32 (exact: |field| < 2^21).
// Each field is taken out with 32-bit shifts (a 3D field may straddle the two
// halves of the word), so the conversion is a 32-bit one.
template <int D>
__device__ inline float fix_field(typename FixPack<D>::word w, int j)
{
    constexpr int b = FixPack<D>::kBits;
    const uint32_t x = (uint32_t)(w >> (b * j));
    return (float)((int32_t)(x << (32 - b)) >> (32 - b));
}

// ------------------------------------------------------------------ helpers
// Lanes of the wave for which p holds (the condition's own lane mask, with
// no detour through a 0/1 register).
__device__ inline unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, kWave); }

__device__ inline long long shfl_xor_ll(long long v, int m) { return __shfl_xor(v, m, kWave); }

// Order-preserving map of doubles to unsigned 64-bit integers, so that the
// integer atomicMin/atomicMax of the encoding are the exact FP64 min/max.
__device__ inline unsigned long long enc_ord(double x)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b & 0x8000000000000000ULL) ? ~b : (b | 0x8000000000000000ULL);
}

__host__ __device__ inline double dec_ord(unsigned long long e)
{
    unsigned long long b = (e & 0x8000000000000000ULL) ? (e & 0x7FFFFFFFFFFFFFFFULL) : ~e;
    union { unsigned long long u; double d; } v;
    v.u = b;
    return v.d;
}

// The FP32 screen's squared inverse influence: 1/I rounded to FP32, squared
// in FP32.
__device__ inline float screen_w2(double iv)
{
    const float fi = (float)iv;
    return fi * fi;
}

// Smallest two values of a set (a <= b), merged pairwise.
struct Two { double a, b; };

__device__ inline Two merge_two(Two x, Two y)
{
    Two r;
    r.a = fmin(x.a, y.a);
    r.b = fmin(fmax(x.a, y.a), fmin(x.b, y.b));
    return r;
}

__device__ inline Two wave_two(Two t)
{
    for (int m = kWave / 2; m > 0; m >>= 1) {
        Two o;
        o.a = shfl_xor_d(t.a, m);
        o.b = shfl_xor_d(t.b, m);
        t = merge_two(t, o);
    }
    return t;
}

__device__ inline double wave_max_d(double v)
{
    for (int m = kWave / 2; m > 0; m >>= 1) v = fmax(v, shfl_xor_d(v, m));
    return v;
}

__device__ inline double wave_min_d(double v)
{
    for (int m = kWave / 2; m > 0; m >>= 1) v = fmin(v, shfl_xor_d(v, m));
    return v;
}

__device__ inline double wave_sum_d(double v)
{
    for (int m = kWave / 2; m > 0; m >>= 1) v += shfl_xor_d(v, m);
    return v;
}

__device__ inline long long wave_sum_ll(long long v)
{
    for (int m = kWave / 2; m > 0; m >>= 1) v += shfl_xor_ll(v, m);
    return v;
}

// Lane-shift of a 64-bit value through the data-parallel-primitive network
// (row shifts within rows of 16 lanes, then the row-15 and row-31
// broadcasts); lanes the pattern does not feed get 0 and must not use it.
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_u64(unsigned long long v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), CTRL, ROWS, 0xf, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Reductions of FP64 values over the wave through the same network: an
// inclusive scan whose last lane holds the result, read back as a
// wave-uniform value.  `idle` is the neutral element the network feeds to
// lanes without a source.
template <int CTRL, int ROWS>
__device__ inline double dpp_d(double v, double idle)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned long long z = (unsigned long long)__double_as_longlong(idle);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)z, (int)(unsigned)u, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(z >> 32), (int)(unsigned)(u >> 32), CTRL,
                                               ROWS, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double readlane_last_d(double v)
{
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, kWave - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), kWave - 1);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Largest of N values per lane over the wave (the reductions interleaved),
// wave-uniform.
template <int CTRL, int ROWS, int N>
__device__ inline void max_step_dpp(double* v)
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = fmax(v[i], dpp_d<CTRL, ROWS>(v[i], -INFINITY));
}

template <int N>
__device__ inline void wave_max_dpp(double* v)
{
    max_step_dpp<0x111, 0xf, N>(v);   // row_shr:1
    max_step_dpp<0x112, 0xf, N>(v);   // row_shr:2
    max_step_dpp<0x114, 0xf, N>(v);   // row_shr:4
    max_step_dpp<0x118, 0xf, N>(v);   // row_shr:8
    max_step_dpp<0x142, 0xa, N>(v);   // row_bcast:15
    max_step_dpp<0x143, 0xc, N>(v);   // row_bcast:31
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = readlane_last_d(v[i]);
}

template <int CTRL, int ROWS>
__device__ inline Two two_step_dpp(Two t)
{
    const Two o{dpp_d<CTRL, ROWS>(t.a, INFINITY), dpp_d<CTRL, ROWS>(t.b, INFINITY)};
    return merge_two(t, o);
}

// The two smallest values over the wave (as wave_two), wave-uniform.
__device__ inline Two wave_two_dpp(Two t)
{
    t = two_step_dpp<0x111, 0xf>(t);
    t = two_step_dpp<0x112, 0xf>(t);
    t = two_step_dpp<0x114, 0xf>(t);
    t = two_step_dpp<0x118, 0xf>(t);
    t = two_step_dpp<0x142, 0xa>(t);
    t = two_step_dpp<0x143, 0xc>(t);
    return Two{readlane_last_d(t.a), readlane_last_d(t.b)};
}

// Sum of a 64-bit integer over the wave, returned on every lane: an
// inclusive scan through the shift network (VALU only, no LDS), whose last
// lane holds the total.
__device__ inline long long wave_sum_dpp(long long v)
{
    const int lane = threadIdx.x % kWave;
    const int rl = lane & 15, row = lane >> 4;
    unsigned long long u = (unsigned long long)v, o;
    o = dpp_u64<0x111, 0xf>(u); u += rl >= 1 ? o : 0ULL;
    o = dpp_u64<0x112, 0xf>(u); u += rl >= 2 ? o : 0ULL;
    o = dpp_u64<0x114, 0xf>(u); u += rl >= 4 ? o : 0ULL;
    o = dpp_u64<0x118, 0xf>(u); u += rl >= 8 ? o : 0ULL;
    o = dpp_u64<0x142, 0xa>(u); u += (row & 1) ? o : 0ULL;
    o = dpp_u64<0x143, 0xc>(u); u += row >= 2 ? o : 0ULL;
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, kWave - 1);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), kWave - 1);
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Fixed-point pair (hi, lo) of a non-negative FP64 value already scaled so
// that it is below 2^61.
__device__ inline void fix_split(double scaled, long long& hi, long long& lo)
{
    long long q = __double2ll_rn(scaled);
    hi = q >> kFixShift;
    lo = q & kFixLoMask;
}

__host__ __device__ inline double fix_value(long long hi, long long lo)
{
    return (double)hi * (double)(1LL << kFixShift) + (double)lo;
}

// Directed conversions FP64 -> FP32.
__device__ inline float f32_up(double x) { return __double2float_ru(x); }
__device__ inline float f32_down(double x) { return __double2float_rd(x); }

// The sweep's copies of the lower-bound frame (M, E): FP32 values rounded so
// that every bound stays valid, and the reciprocal of M (its rounding, a few
// units of 2^-53, is covered by the sweep's 1e-12 slack).  Called by the one
// thread that has just changed M or E.
// One relaxation step of a tile's lower-bound frame: m, e the smallest ratio
// and largest shift over its candidates, lb_out the bound on the rest.
__device__ inline void tile_bound_step(TileBound& f, double m, double e, double lb_out)
{
    f.M = f.M * m * (1.0 - 0x1p-50);
    f.E = (f.E * m + e) * (1.0 + 0x1p-50);
    f.Mf = f32_down(f.M);
    f.Ef = f32_up(f.E);
    f.Edn = f32_down(f.E);
    f.invMdn = f32_down((1.0 / f.M) * (1.0 - 0x1p-21));
    f.lam = f32_down((lb_out + f.E) / f.M * (1.0 - 0x1p-50));
}

__device__ inline void frame_copies(DevState* st)
{
    st->Mf = f32_down(st->M);
    st->Ef = f32_up(st->E);
    st->invM = 1.0 / st->M;
    st->Edn = f32_down(st->E);
    st->invMdn = f32_down(st->invM * (1.0 - 0x1p-21));
}

// ------------------------------------------------------------- launchers
// Each returns the hipError_t of its last launch.

hipError_t launch_bbox(const RunDev& r, int hilbert_order, hipStream_t s);
hipError_t launch_keys(const RunDev& r, int hilbert_order, int32_t* vals, hipStream_t s);
hipError_t radix_sort_pairs(const RunDev& r, uint64_t* keys, int32_t* vals, int nbits,
                            hipStream_t s);
hipError_t launch_permute(const RunDev& r, hipStream_t s);
hipError_t launch_jump_plan(const RunDev& r, hipStream_t s);
hipError_t launch_place(const RunDev& r, hipStream_t s);
hipError_t launch_tile_prep(const RunDev& r, hipStream_t s);
hipError_t launch_centers_from_sorted(const RunDev& r, double* out, int row_major,
                                      hipStream_t s);
hipError_t launch_target_prep(const RunDev& r, double eps, hipStream_t s);
hipError_t launch_init_run(const RunDev& r, const double* centers_init_rowmajor,
                           const double* influence_init, int max_iter, int max_balance_iter,
                           double eps, double delta_threshold, hipStream_t s);
// random-sample initialization: order of the points by (key, index), keys from
// splitmix64 or given (in sperm); then the rank of the point at every layout
// position, and per sample the layout positions of rank below `count`, in
// layout order, with their coordinates and weights
hipError_t launch_sample_order(const RunDev& r, uint64_t seed, const uint64_t* given,
                               hipStream_t s);
hipError_t launch_sample_layout_rank(const RunDev& r, int32_t* rank, int32_t* rk, hipStream_t s);
hipError_t launch_sample_compact(const RunDev& r, const int32_t* rk, int64_t count, void* const* x,
                                 double* w, hipStream_t s);
hipError_t launch_iota(int32_t* v, int64_t n, hipStream_t s);
hipError_t launch_supercand(const RunDev& r, hipStream_t s);
hipError_t launch_tilecand(const RunDev& r, hipStream_t s);
hipError_t launch_sweep(const RunDev& r, hipStream_t s);
hipError_t launch_balance(const RunDev& r, hipStream_t s);
hipError_t launch_block_boxes(const RunDev& r, hipStream_t s);

// Instances of one class (same d, precision, tile size and weighting) whose
// per-sweep kernels run as one launch each.  The maps give, for every block
// of a launch, its instance and its block within that instance.
struct MultiSet {
    int d, precision, ppt, weighted;
    int ninst;
    const RunDev* rs;          // device [ninst]
    const int2* map_super;     // one block per super-tile
    const int2* map_quad;      // one block per 4 tiles (a wave per tile)
    const int2* map_tile;      // one block per tile
    const int2* map_pass;      // one block per kPassGroups groups
    const int2* map_inst;      // one block per instance
    const int2* map_hyper;     // one block per hyper-tile
    int nb_super, nb_quad, nb_tile, nb_pass, nb_hyper;
};
constexpr int kPassGroupsHost = 256;   // groups per block of the round-end pass
hipError_t launch_sweep_multi(const MultiSet& m, hipStream_t s);    // candidates + sweep
hipError_t launch_update_multi(const MultiSet& m, hipStream_t s);   // balance + round end + move
hipError_t launch_move(const RunDev& r, hipStream_t s);
// debug checks of the stored bounds (and, after a sweep, the block) of every
// debug_stride-th point against a brute-force FP64 evaluation; after_sweep
// selects the check of the block as the argmin
hipError_t launch_check_bounds(const RunDev& r, int after_sweep, hipStream_t s);
hipError_t launch_set_step(const RunDev& r, const double* centers_rm, const double* infl,
                           int first, hipStream_t s);
hipError_t launch_finish(const RunDev& r, int32_t* assignment_out, double* centers_out,
                         double* influence_out, double* bw_out, hipStream_t s);
hipError_t launch_stats(const RunDev& r, const int32_t* assignment, double eps,
                        double* bw_out, double* centers_out, double* out6, hipStream_t s);

}  // namespace bkm
