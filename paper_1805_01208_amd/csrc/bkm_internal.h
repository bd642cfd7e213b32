// Internal declarations of libbkm: device state, the device-memory layout of one
// run, launch wrappers and wave-level helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bkm.h"

namespace bkm {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per block of the point kernels
constexpr int kLcap = 1024;          // super-tile candidates a tile can stage
constexpr int kMaxc = 256;           // tile candidates held in LDS per chunk
constexpr int kFixShift = 30;        // fixed-point sums: term = hi * 2^30 + lo
constexpr long long kFixLoMask = (1LL << kFixShift) - 1;

// Control and scalar state of one run, resident in device memory.  Kernels
// of a round read it to decide whether they still have work (a finished
// AssignAndBalance call or a finished run turns later launches into no-ops),
// so the host only synchronises once per round.
struct DevState {
    int32_t done;             // run finished (converged or out of rounds)
    int32_t round_done;       // current AssignAndBalance call finished
    int32_t balanced;         // result of the last balance test
    int32_t converged;
    int32_t rounds;           // AssignAndBalance calls completed
    int32_t sweep_in_round;   // sweeps made in the current call
    int32_t sweeps;           // sweeps made in total
    int32_t max_iter;
    int32_t max_balance_iter;
    int32_t bad_data;         // a non-finite coordinate or a bad weight was seen
    int32_t nonempty;         // non-empty blocks seen by the last center update
    int32_t pad;
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
    unsigned long long evaluated, skipped, rechecked, changed, cand_evals, overflow_tiles;
};

// Everything a run keeps on the device.  Point arrays are in Hilbert (sorted)
// order and padded to whole tiles.
struct RunDev {
    int64_t n, npad;
    int d, k, in_f32, weighted;
    int T, ppt, ntiles, super_tiles, nsuper, ngroups;
    int precision, use_bounds;
    double recheck_gap;

    const void* in_x[3];      // caller's coordinates (input order)
    const double* in_w;       // caller's weights or null

    double* xs64[3];          // sorted master coordinates (FP64 input)
    float* xs32[3];           // sorted master coordinates (FP32 input)
    float* ofs[3];            // FP32 offsets from the tile anchor (FP32 sweep)
    double* ws;               // sorted weights or null
    int32_t* perm;            // sorted position -> input index
    int32_t* A;               // current block of each sorted point (-1: none yet)
    float* ubt;               // stored upper bounds (distance frame)
    float* lbt;               // stored lower bounds (lazy frame)
    double* tbox;             // [ntiles][2d] lo..., hi...
    double* gbox;             // [ngroups][2d] boxes of 64-point groups
    double* sbox;             // [nsuper][2d]
    int32_t* slist;           // [nsuper][k] candidate centers of each super-tile
    int32_t* scount;          // [nsuper]
    double* C;                // [d][k] centers (SoA)
    double* I;                // [k] influence
    double2* clus;            // [k] (accumulated movement, 1/influence)
    long long* acc;           // [k][kAcc] fixed-point block sums
    unsigned long long* bb;   // [k][2d] encoded block boxes (min..., max...)
    DevState* st;
    // bootstrap scratch
    uint64_t* keys;
    uint64_t* keys2;
    int32_t* vals2;
    uint32_t* hist;
    uint32_t* part;
    double* red;              // per-block partial reductions
};

// Number of fixed-point accumulators per block: coordinate hi/lo per axis and
// weight hi/lo (count in the hi word for unit weights).
constexpr int kAcc = 8;

// ------------------------------------------------------------------ helpers
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

// ------------------------------------------------------------- launchers
// Each returns the hipError_t of its last launch.
hipError_t launch_bbox(const RunDev& r, int hilbert_order, hipStream_t s);
hipError_t launch_keys(const RunDev& r, int hilbert_order, int32_t* vals, hipStream_t s);
hipError_t radix_sort_pairs(const RunDev& r, uint64_t* keys, int32_t* vals, int nbits,
                            hipStream_t s);
hipError_t launch_permute(const RunDev& r, const int32_t* perm_sorted, hipStream_t s);
hipError_t launch_tile_prep(const RunDev& r, hipStream_t s);
hipError_t launch_centers_from_sorted(const RunDev& r, double* out, int row_major,
                                      hipStream_t s);
hipError_t launch_init_run(const RunDev& r, const double* centers_init_rowmajor,
                           int max_iter, int max_balance_iter, double eps,
                           double delta_threshold, hipStream_t s);
hipError_t launch_supercand(const RunDev& r, hipStream_t s);
hipError_t launch_sweep(const RunDev& r, hipStream_t s);
hipError_t launch_balance(const RunDev& r, hipStream_t s);
hipError_t launch_block_boxes(const RunDev& r, hipStream_t s);
hipError_t launch_move(const RunDev& r, hipStream_t s);
hipError_t launch_set_step(const RunDev& r, const double* centers_rm, const double* infl,
                           int first, hipStream_t s);
hipError_t launch_finish(const RunDev& r, int32_t* assignment_out, double* centers_out,
                         double* influence_out, double* bw_out, hipStream_t s);
hipError_t launch_stats(const RunDev& r, const int32_t* assignment, double eps,
                        double* bw_out, double* centers_out, double* out6, hipStream_t s);

}  // namespace bkm
