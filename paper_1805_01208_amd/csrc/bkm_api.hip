// C ABI of libbkm (include/bkm.h): argument checks, device workspace, and the
// host driver of the SFC bootstrap and the round loop of balanced k-means
// (Alg. 2 around Alg. 1).
//
// The round loop keeps the host out of the per-sweep decision: sweeps,
// balance tests and the round-end kernels read the run's device state and turn
// into no-ops once their AssignAndBalance call (or the run) is over, so the
// host enqueues a batch (one sweep, its balance test and the round end) and
// synchronises once per batch.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bkm_graph_internal.h"
#include "bkm_internal.h"

using namespace bkm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? BKM_ENOMEM : BKM_EHIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                         \
    } while (0)

// Device workspace carved from one stream-ordered allocation.
struct Arena {
    char* base = nullptr;
    size_t off = 0;
    size_t cap = 0;
    hipStream_t s = nullptr;

    template <typename T>
    T* take(size_t count)
    {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        T* p = (T*)(base + off);
        off += bytes;
        return p;
    }
    ~Arena()
    {
        if (base) {
            (void)hipFreeAsync(base, s);
            (void)hipStreamSynchronize(s);
        }
    }
};

struct Sizes {
    size_t total = 0;
    template <typename T>
    void add(size_t count) { total += (count * sizeof(T) + 255) & ~size_t(255); }
};

// Static workspace of the no-allocation entry points: every device the
// library runs on holds one copy until the process ends.  Host code never
// uses the symbol itself as an address (on the host it is only a stand-in):
// its device address is looked up once per device and kept.
static __device__ __align__(256) unsigned char scratch[BKM_NOALLOC_SCRATCH_BYTES];

int scratch_address(char** out)
{
    static std::atomic<char*> addr[64];
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(BKM_EINVAL, "device %d outside [0, 64)", dev);
    char* p = addr[dev].load(std::memory_order_acquire);
    if (!p) {
        HIPCHK(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(BKM_EHIP, "hipGetSymbolAddress returned NULL");
        addr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return BKM_OK;
}

// Keep freed stream-ordered memory in the current device's default pool
// (set once per device; devices 0..63).
void keep_pool_memory()
{
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    const uint64_t bit = uint64_t(1) << dev;
    if (done.load(std::memory_order_relaxed) & bit) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr) == hipSuccess)
            done.fetch_or(bit, std::memory_order_relaxed);
    }
}

// Small pinned host buffer for per-round state reads.
DevState* host_state()
{
    thread_local DevState* h = nullptr;
    if (!h) {
        if (hipHostMalloc((void**)&h, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
            h = nullptr;
    }
    return h;
}

// Pinned two-entry ring the round loop copies the state records into (one
// per thread, kept for the process: pinned allocations are slow).
DevState* loop_ring()
{
    thread_local DevState* h = nullptr;
    if (!h) {
        if (hipHostMalloc((void**)&h, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
            h = nullptr;
    }
    return h;
}

int check_points(const bkm_points* pts)
{
    if (!pts) return fail(BKM_EINVAL, "points is NULL");
    if (pts->n < 1 || pts->n >= (int64_t(1) << 31))
        return fail(BKM_EINVAL, "n = %lld outside [1, 2^31)", (long long)pts->n);
    if (pts->d != 2 && pts->d != 3) return fail(BKM_EINVAL, "d = %d is not 2 or 3", pts->d);
    if (pts->dtype != BKM_F32 && pts->dtype != BKM_F64)
        return fail(BKM_EINVAL, "dtype = %d unknown", pts->dtype);
    for (int j = 0; j < pts->d; ++j)
        if (!pts->coords[j]) return fail(BKM_EINVAL, "coords[%d] is NULL", j);
    return BKM_OK;
}

int check_order(int d, int m)
{
    const int mmax = d == 2 ? 31 : 21;
    if (m < 1 || m > mmax)
        return fail(BKM_EINVAL, "hilbert_order %d outside [1, %d] for d = %d", m, mmax, d);
    return BKM_OK;
}

// Tile, super-tile and group counts of a padded layout of npad points.
void set_layout_size(RunDev& r, int64_t npad)
{
    r.npad = npad;
    r.ntiles = (int)(npad / r.T);
    r.nsuper = (r.ntiles + r.super_tiles - 1) / r.super_tiles;
    r.nhyper = (r.nsuper + kHyper - 1) / kHyper;
    r.ngroups = (int)(npad / kWave);
}

// Fill the sizes of a run and lay its arrays out in the arena.
void plan(RunDev& r, const bkm_points* pts, int k, int T, int ST, int precision, int use_bounds,
          double gap)
{
    std::memset(&r, 0, sizeof(r));
    r.n = pts->n;
    r.d = pts->d;
    r.k = k;
    r.in_f32 = pts->dtype == BKM_F32;
    r.weighted = pts->weights != nullptr;
    r.T = T;
    r.ppt = T / kBlock;
    // capacity of the padded layout: at most maxjumps realigned jumps
    r.maxjumps = (int)std::min<int64_t>(kMaxJumps, std::max<int64_t>(1, r.n / (4 * (int64_t)T)));
    r.npad_cap = (r.n + (int64_t)r.maxjumps * (T - 1) + T - 1) / T * T;
    r.super_tiles = ST;
    set_layout_size(r, (r.n + T - 1) / T * T);
    r.precision = precision;
    r.use_bounds = use_bounds;
    r.recheck_gap = gap;
    for (int j = 0; j < r.d; ++j) r.in_x[j] = pts->coords[j];
    r.in_w = pts->weights;
}

size_t layout(RunDev& r, Arena* a, bool full)
{
    Sizes z;
    const int64_t n = r.n, np = r.npad_cap;
    const int64_t ntiles = np / r.T;
    const int64_t nsuper = (ntiles + r.super_tiles - 1) / r.super_tiles;
    const int d = r.d, k = r.k;
    const int nblk = (int)((n + kSortChunk - 1) / kSortChunk);
    const int64_t hlen = (int64_t)256 * nblk;
    const int nseg = (int)((hlen + 1023) / 1024);
    auto both = [&](auto* tag, size_t count, auto*& ptr) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (a)
            ptr = a->take<T>(count);
        else
            z.add<T>(count);
    };
    both((DevState*)nullptr, 1, r.st);
    both((unsigned long long*)nullptr, kCntSlots * kCntWords, r.cnt);
    both((double*)nullptr, std::max<int64_t>(32768, k), r.red);
    both((uint64_t*)nullptr, n, r.keys);
    both((uint64_t*)nullptr, n, r.keys2);
    both((int32_t*)nullptr, n, r.sperm);
    both((int32_t*)nullptr, n, r.vals2);
    both((uint32_t*)nullptr, hlen, r.hist);
    both((uint32_t*)nullptr, nseg + 1, r.part);
    for (int j = 0; j < d; ++j) {
        if (r.in_f32)
            both((float*)nullptr, n, r.tx32[j]);
        else
            both((double*)nullptr, n, r.tx64[j]);
    }
    both((double*)nullptr, (size_t)d * k, r.C);
    if (full) {
        both((unsigned int*)nullptr, kGapBins, r.ghist);
        both((int32_t*)nullptr, r.maxjumps, r.jumps);
        both((int64_t*)nullptr, r.maxjumps, r.jshift);
        both((int32_t*)nullptr, np, r.perm);
        for (int j = 0; j < d; ++j) {
            if (r.in_f32)
                both((float*)nullptr, np, r.xs32[j]);
            else
                both((double*)nullptr, np, r.xs64[j]);
        }
        if (r.precision == BKM_PREC_F32_RECHECK)
            both((uint32_t*)nullptr, (size_t)np * (d == 3 ? 2 : 1), *reinterpret_cast<uint32_t**>(&r.ofs));
        if (r.weighted) both((double*)nullptr, np, r.ws);
        both((int32_t*)nullptr, np, r.A);
        both((float2*)nullptr, np, r.bnd);
        both((double*)nullptr, (size_t)ntiles * 2 * d, r.tbox);
        both((TileFrame*)nullptr, (size_t)ntiles, r.tframe);
        both((TileBound*)nullptr, (size_t)ntiles, r.tbnd);
        both((double2*)nullptr, (size_t)k, r.cdec);
        both((double*)nullptr, (size_t)(np / kWave) * 2 * d, r.gbox);
        const int64_t nhyper = (nsuper + kHyper - 1) / kHyper;
        both((double*)nullptr, (size_t)nhyper * 2 * d, r.hbox);
        both((int32_t*)nullptr, (size_t)nhyper * k, r.hlist);
        both((int32_t*)nullptr, (size_t)nhyper, r.hcount);
        both((double*)nullptr, (size_t)nsuper * 2 * d, r.sbox);
        both((int32_t*)nullptr, (size_t)nsuper * k, r.slist);
        both((int32_t*)nullptr, (size_t)nsuper, r.scount);
        both((TileHead*)nullptr, (size_t)ntiles, r.thead);
        both((CandRec*)nullptr, (size_t)ntiles * kTileCap, r.tcand);
        both((double*)nullptr, (size_t)k, r.I);
        if (r.tsz) {
            both((double*)nullptr, (size_t)k, r.tT);
            both((double*)nullptr, (size_t)k, r.tL);
            both((double*)nullptr, (size_t)k + 1, r.tpre);
        }
        both((double2*)nullptr, (size_t)k, r.clus);
        both((float2*)nullptr, (size_t)k, r.clus32);
        both((float*)nullptr, (size_t)k, r.clusdn);
        both((double*)nullptr, (size_t)k, r.ivb);
        both((int32_t*)nullptr, (size_t)(np / kWave), r.gblk);
        both((int32_t*)nullptr, (size_t)(np / kWave), r.gdirty);
        both((int32_t*)nullptr, np, r.Aprev);
        both((long long*)nullptr, (size_t)k * kAcc, r.acc);
        both((unsigned long long*)nullptr, (size_t)k * 2 * d, r.bb);
    }
    return z.total;
}

int alloc_run(RunDev& r, Arena& a, hipStream_t s, bool full)
{
    size_t bytes = layout(r, nullptr, full);
    a.s = s;
    hipError_t e = hipMallocAsync((void**)&a.base, bytes, s);
    if (e != hipSuccess) {
        a.base = nullptr;
        return fail(e == hipErrorOutOfMemory ? BKM_ENOMEM : BKM_EHIP,
                    "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
    }
    a.cap = bytes;
    layout(r, &a, full);
    HIPCHK(hipMemsetAsync(r.st, 0, sizeof(DevState), s));
    return BKM_OK;
}

int read_state(const RunDev& r, hipStream_t s, DevState* out)
{
    DevState* h = host_state();
    if (!h) return fail(BKM_ENOMEM, "pinned host buffer unavailable");
    HIPCHK(hipMemcpyAsync(h, r.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = *h;
    return BKM_OK;
}

int read_counters(const RunDev& r, hipStream_t s, unsigned long long out[kCntWords])
{
    unsigned long long h[kCntSlots * kCntWords];
    HIPCHK(hipMemcpyAsync(h, r.cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int j = 0; j < kCntWords; ++j) {
        out[j] = 0;
        for (int q = 0; q < kCntSlots; ++q) out[j] += h[q * kCntWords + j];
    }
    return BKM_OK;
}

// SFC bootstrap: bounding box (+ data checks), keys, sort, coordinates in
// Hilbert order; with `tiles`, also the jump-aligned padded layout and the
// tile, group and super-tile boxes.
// presorted: the points already come in a spatially coherent order (a sample
// taken from a Hilbert layout), which is kept instead of sorting by key.
int bootstrap(RunDev& r, int order, hipStream_t s, bool tiles, double eps = 0.0,
              bool presorted = false)
{
    HIPCHK(launch_bbox(r, order, s));
    if (r.tsz) HIPCHK(launch_target_prep(r, eps, s));
    DevState h;
    int rc = read_state(r, s, &h);
    if (rc) return rc;
    if (h.bad_data & 4)
        return fail(BKM_EINVAL, "target_sizes must be finite and > 0, with a finite sum");
    if (h.bad_data)
        return fail(BKM_EDATA, r.weighted ? "non-finite coordinate or weight <= 0 / non-finite"
                                          : "non-finite coordinate");
    if (presorted) {
        HIPCHK(launch_iota(r.sperm, r.n, s));
    } else {
        HIPCHK(launch_keys(r, order, r.sperm, s));
        HIPCHK(radix_sort_pairs(r, r.keys, r.sperm, r.d * order, s));
    }
    HIPCHK(launch_permute(r, s));
    if (!tiles) return BKM_OK;
    HIPCHK(launch_jump_plan(r, s));
    if ((rc = read_state(r, s, &h))) return rc;
    if (h.npad < r.n || h.npad > r.npad_cap)
        return fail(BKM_EHIP, "padded layout of %lld points outside [n, %lld]", (long long)h.npad,
                    (long long)r.npad_cap);
    set_layout_size(r, h.npad);
    HIPCHK(launch_place(r, s));
    HIPCHK(launch_tile_prep(r, s));
    return BKM_OK;
}

int check_tile(int T) { return T == -1 || T == 0 || T == 256 || T == 512 || T == 1024; }

// Arguments of one balanced k-means run.
int check_run(const bkm_points* pts, const bkm_params* prm)
{
    int rc = check_points(pts);
    if (rc) return rc;
    if (!prm) return fail(BKM_EINVAL, "params is NULL");
    const bkm_params& p = *prm;
    if (p.k < 1 || p.k > pts->n) return fail(BKM_EINVAL, "k = %d outside [1, n]", p.k);
    if (!(p.epsilon >= 0.0)) return fail(BKM_EINVAL, "epsilon must be >= 0");
    if (p.max_iter < 1 || p.max_balance_iter < 1)
        return fail(BKM_EINVAL, "max_iter and max_balance_iter must be >= 1");
    if ((rc = check_order(pts->d, p.hilbert_order))) return rc;
    if (p.precision != BKM_PREC_F64 && p.precision != BKM_PREC_F32_RECHECK)
        return fail(BKM_EINVAL, "precision %d unknown", p.precision);
    if (!check_tile(p.tile_points))
        return fail(BKM_EINVAL, "tile_points %d not -1/0/256/512/1024", p.tile_points);
    if (p.super_tiles < 0) return fail(BKM_EINVAL, "super_tiles must be >= 0");
    if (!(p.recheck_rel_gap >= 0.0) || !std::isfinite(p.recheck_rel_gap))
        return fail(BKM_EINVAL, "recheck_rel_gap must be finite and >= 0");
    if (std::isnan(p.delta_threshold)) return fail(BKM_EINVAL, "delta_threshold is NaN");
    if (p.sample_init && p.sample_start < 0) return fail(BKM_EINVAL, "sample_start must be >= 0");
    if (p.erosion != 0 && p.erosion != 1) return fail(BKM_EINVAL, "erosion must be 0 or 1");
    if (p.debug_checks < 0 || p.debug_checks > 2)
        return fail(BKM_EINVAL, "debug_checks must be 0, 1 or 2");
    return BKM_OK;
}

// Tile size for tile_points = -1, from the mean number of points per block:
// smaller blocks want smaller tiles, whose boxes keep fewer candidates.
int auto_tile(int64_t n, int k)
{
    const double ppb = (double)n / (double)k;
    return ppb >= 2048.0 ? 1024 : ppb >= 512.0 ? 512 : 256;
}

void fill_info(bkm_info* info, const DevState& h, const unsigned long long* cnt)
{
    std::memset(info, 0, sizeof(*info));
    info->rounds = h.rounds;
    info->sweeps = h.sweeps;
    info->balanced = h.balanced;
    info->converged = h.converged;
    info->l_max = h.lmax;
    info->max_block_weight = h.max_weight;
    info->imbalance = h.max_ratio - 1.0;
    info->evaluated = (int64_t)cnt[kCntEvaluated];
    info->skipped = (int64_t)cnt[kCntSkipped];
    info->rechecked = (int64_t)cnt[kCntRechecked];
    info->changed = (int64_t)cnt[kCntChanged];
    info->candidate_evals = (int64_t)cnt[kCntCandEvals];
    info->overflow_tiles = (int64_t)cnt[kCntOverflow];
    info->debug_checked = (int64_t)cnt[kCntDebugChecked];
    info->debug_violations = (int64_t)cnt[kCntDebugViolated];
    info->list_builds = (int64_t)cnt[kCntListBuilds];
}

// Owned HIP objects of a batched call, released on every return path.
struct BatchRes {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    DevState* hstates = nullptr;
    unsigned long long* hcnt = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchRes()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto e : events) (void)hipEventDestroy(e);
        for (auto q : streams) {
            (void)hipStreamSynchronize(q);
            (void)hipStreamDestroy(q);
        }
        if (hstates) (void)hipHostFree(hstates);
        if (hcnt) (void)hipHostFree(hcnt);
    }
};

int run_core(const bkm_points* pts, const bkm_params& p, const double* centers_init,
             const double* influence_init, int32_t* assignment_out, double* centers_out,
             double* influence_out, double* block_weights_out, bkm_info* info, hipStream_t s,
             bool presorted = false);

// ------------------------------------------------------------- autotuner
// Tile size and tiles per super-tile of the sweep, chosen by measurement.
// A configuration is timed by short balanced k-means runs (kTuneRounds
// rounds, twice, the faster counts) on a strided sample of at most
// kTuneSample points with k scaled to keep the mean points per block; the
// objective is the device time of the candidate filters and the sweep per
// sweep.  Choices are cached per (device architecture, d, precision,
// weighting, octave of n/k, size class of n: below 2^17, 2^20, 2^23, above),
// in the process and, when the environment names a file in BKM_TUNE_CACHE,
// in that file (one line per key, read once, appended on every new entry).
constexpr int kTuneTiles[] = {256, 512, 1024};
constexpr int kTuneSupers[] = {8, 16, 24, 32};
constexpr int64_t kTuneSample = int64_t(1) << 23;
constexpr int kTuneRounds = 3;

struct TuneEntry {
    int T, ST;
    double us;
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const bkm_points* pts, const bkm_params& p)
{
    int dev = 0;
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch = arch.substr(0, c);
    }
    const int ppb = (int)std::lround(std::log2((double)pts->n / (double)p.k));
    const int nb = pts->n < (int64_t(1) << 17) ? 0 : pts->n < (int64_t(1) << 20) ? 1
                 : pts->n < kTuneSample ? 2 : 3;
    char buf[160];
    snprintf(buf, sizeof(buf), "%s d%d p%d w%d ppb%d n%d", arch.c_str(), pts->d, p.precision,
             pts->weights ? 1 : 0, ppb, nb);
    return buf;
}

// Reads the cache file once (lines "key... | T ST us"); the mutex is held.
void tune_load_locked()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("BKM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof(line), f)) {
        char* bar = std::strchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        std::string key(line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        TuneEntry e;
        if (std::sscanf(bar + 1, "%d %d %lf", &e.T, &e.ST, &e.us) == 3 && check_tile(e.T) &&
            e.T > 0 && e.ST >= 1)
            g_tune[key] = e;
    }
    std::fclose(f);
}

void tune_store_locked(const std::string& key, const TuneEntry& e)
{
    g_tune[key] = e;
    const char* path = std::getenv("BKM_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s | %d %d %.3f\n", key.c_str(), e.T, e.ST, e.us);
    std::fclose(f);
}

// Device time per sweep of the candidate filters and the sweep for one
// configuration on the sample (the faster of two short runs).
int tune_time(const bkm_points* ps, const bkm_params& p, int T, int ST, int32_t* abuf,
              double* cbuf, hipStream_t s, double* us)
{
    bkm_params q = p;
    q.tile_points = T;
    q.super_tiles = ST;
    q.timing = 1;
    q.sample_init = 0;
    q.target_sizes = nullptr;
    q.max_iter = kTuneRounds;
    *us = INFINITY;
    for (int rep = 0; rep < 2; ++rep) {
        bkm_info info;
        const int rc = run_core(ps, q, nullptr, nullptr, abuf, cbuf, nullptr, nullptr, &info, s);
        if (rc < 0) return rc;
        if (info.sweeps > 0)
            *us = std::min(*us, 1e3 * (info.cand_ms + info.sweep_ms) / info.sweeps);
    }
    return BKM_OK;
}

// Measures every configuration on a strided sample of the points.
int tune_measure(const bkm_points* pts, const bkm_params& p, hipStream_t s, TuneEntry* best,
                 bkm_tune_result* res)
{
    const int64_t n = pts->n;
    const int64_t stride = std::max<int64_t>(1, (n + kTuneSample - 1) / kTuneSample);
    const int64_t ns = (n + stride - 1) / stride;
    const int ks = (int)std::max<int64_t>(1, std::min<int64_t>(ns, std::llround((double)p.k * ns / n)));
    const size_t es = pts->dtype == BKM_F32 ? sizeof(float) : sizeof(double);
    Sizes z;
    for (int j = 0; j < pts->d; ++j) z.add<char>((size_t)ns * es);
    if (pts->weights) z.add<double>((size_t)ns);
    z.add<int32_t>((size_t)ns);
    z.add<double>((size_t)ks * pts->d);
    Arena a;
    a.s = s;
    HIPCHK(hipMallocAsync((void**)&a.base, z.total, s));
    bkm_points ps = *pts;
    ps.n = ns;
    for (int j = 0; j < pts->d; ++j) {
        char* dst = a.take<char>((size_t)ns * es);
        HIPCHK(hipMemcpy2DAsync(dst, es, pts->coords[j], es * stride, es, ns,
                                hipMemcpyDeviceToDevice, s));
        ps.coords[j] = dst;
    }
    if (pts->weights) {
        double* w = a.take<double>((size_t)ns);
        HIPCHK(hipMemcpy2DAsync(w, sizeof(double), pts->weights, sizeof(double) * stride,
                                sizeof(double), ns, hipMemcpyDeviceToDevice, s));
        ps.weights = w;
    }
    int32_t* abuf = a.take<int32_t>((size_t)ns);
    double* cbuf = a.take<double>((size_t)ks * pts->d);
    bkm_params q = p;
    q.k = ks;
    best->us = INFINITY;
    best->T = auto_tile(n, p.k);
    best->ST = 16;
    int timed = 0;
    double def_us = 0.0;
    for (int T : kTuneTiles) {
        for (int ST : kTuneSupers) {
            double us;
            const int rc = tune_time(&ps, q, T, ST, abuf, cbuf, s, &us);
            if (rc < 0) return rc;
            ++timed;
            if (T == auto_tile(n, p.k) && ST == 16) def_us = us;
            if (us < best->us) *best = TuneEntry{T, ST, us};
        }
    }
    if (res) {
        res->candidates = timed;
        res->default_us = def_us;
        res->sample_points = ns;
        res->sample_k = ks;
    }
    return BKM_OK;
}

// The tuned configuration for these points and parameters: from the cache,
// or measured now (and cached).
int tuned_tiles(const bkm_points* pts, const bkm_params& p, hipStream_t s, int* T, int* ST,
                bkm_tune_result* res, bool force = false)
{
    const std::string key = tune_key(pts, p);
    if (res) std::memset(res, 0, sizeof(*res));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (!force && it != g_tune.end()) {
            *T = it->second.T;
            *ST = p.super_tiles ? p.super_tiles : it->second.ST;
            if (res) {
                res->tile_points = *T;
                res->super_tiles = *ST;
                res->from_cache = 1;
                res->best_us = it->second.us;
            }
            return BKM_OK;
        }
    }
    TuneEntry e;
    const int rc = tune_measure(pts, p, s, &e, res);
    if (rc < 0) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_store_locked(key, e);
    }
    *T = e.T;
    *ST = p.super_tiles ? p.super_tiles : e.ST;
    if (res) {
        res->tile_points = *T;
        res->super_tiles = *ST;
        res->from_cache = 0;
        res->best_us = e.us;
    }
    return BKM_OK;
}

// One balanced k-means run (Alg. 2 around Alg. 1) on checked arguments.
// centers_init ([k][d]) and influence_init ([k]) may be NULL (SFC centers,
// influence 1); with centers given, k may exceed n (a sample round).
// presorted: the points come in Hilbert order already (a sample round).
int run_core(const bkm_points* pts, const bkm_params& p, const double* centers_init,
             const double* influence_init, int32_t* assignment_out, double* centers_out,
             double* influence_out, double* block_weights_out, bkm_info* info, hipStream_t s,
             bool presorted)
{
    int rc;
    int T = p.tile_points > 0 ? p.tile_points : auto_tile(pts->n, p.k);
    int ST = p.super_tiles ? p.super_tiles : 16;
    if (p.tile_points == 0 && (rc = tuned_tiles(pts, p, s, &T, &ST, nullptr)) < 0) return rc;
    RunDev r;
    plan(r, pts, p.k, T, ST, p.precision, p.use_bounds ? 1 : 0, p.recheck_rel_gap);
    r.tsz = p.target_sizes;
    r.erosion = p.erosion;
    // debug checks: every point, or a stride that keeps a check near 2^26
    // point-center pairs
    if (p.debug_checks == 2)
        r.debug_stride = 1;
    else if (p.debug_checks == 1)
        r.debug_stride = (int)std::max<int64_t>(1, ((int64_t)r.npad_cap * p.k) >> 26);
    Arena a;
    if ((rc = alloc_run(r, a, s, true))) return rc;

    hipEvent_t ev[3];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    struct EvFree { hipEvent_t* e; ~EvFree() { for (int i = 0; i < 3; ++i) (void)hipEventDestroy(e[i]); } } evf{ev};
    HIPCHK(hipEventRecord(ev[0], s));

    if ((rc = bootstrap(r, p.hilbert_order, s, true, p.epsilon, presorted))) return rc;

    // random-sample initialization: rounds on the first sz points of a random
    // order, sz doubling, each one AssignAndBalance and one center movement
    // with erosion on the sample alone (its own balance target), carrying
    // centers and influence on; the delta threshold is that of all points
    int32_t sample_rounds = 0, sample_sweeps = 0;
    const double* cinit = centers_init;
    const double* iinit = influence_init;
    double dthr = p.delta_threshold;
    Arena sa;
    // first sample size: sample_start, or 0 for 100 points per block (the
    // paper's 100 points per process, with one block per process)
    const int64_t s0 = p.sample_start > 0 ? p.sample_start : 100 * (int64_t)p.k;
    if (p.sample_init && s0 < pts->n) {
        DevState h0;
        if ((rc = read_state(r, s, &h0))) return rc;
        if (dthr < 0.0) dthr = 1e-5 * h0.ext;
        const int64_t n = pts->n;
        Sizes z;
        z.add<double>((size_t)p.k * r.d);
        z.add<double>((size_t)p.k);
        z.add<int32_t>((size_t)n);
        for (int j = 0; j < r.d; ++j) z.add<double>((size_t)n);   // room for either dtype
        if (r.weighted) z.add<double>((size_t)n);
        z.add<int32_t>((size_t)n);         // rank of each point in the random order
        z.add<int32_t>((size_t)r.npad);    // rank of the point at each layout position
        sa.s = s;
        HIPCHK(hipMallocAsync((void**)&sa.base, z.total, s));
        sa.cap = z.total;
        double* cbuf = sa.take<double>((size_t)p.k * r.d);
        double* ibuf = sa.take<double>((size_t)p.k);
        int32_t* abuf = sa.take<int32_t>((size_t)n);
        void* xb[3] = {nullptr, nullptr, nullptr};
        for (int j = 0; j < r.d; ++j) xb[j] = sa.take<double>((size_t)n);
        double* wb = r.weighted ? sa.take<double>((size_t)n) : nullptr;
        int32_t* rank = sa.take<int32_t>((size_t)n);
        int32_t* rk = sa.take<int32_t>((size_t)r.npad);
        if (centers_init)
            HIPCHK(hipMemcpyAsync(cbuf, centers_init, (size_t)p.k * r.d * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        else
            HIPCHK(launch_centers_from_sorted(r, cbuf, 1, s));
        if (influence_init)
            HIPCHK(hipMemcpyAsync(ibuf, influence_init, (size_t)p.k * sizeof(double),
                                  hipMemcpyDeviceToDevice, s));
        HIPCHK(launch_sample_order(r, p.seed, p.sample_keys, s));
        HIPCHK(launch_sample_layout_rank(r, rank, rk, s));
        bkm_params q = p;
        q.sample_init = 0;
        q.max_iter = 1;
        // the short sample rounds take the n/k rule rather than tuning
        // every sample size
        if (q.tile_points == 0) q.tile_points = -1;
        q.delta_threshold = dthr;
        q.timing = 0;
        for (int64_t sz = s0; sz < n; sz *= 2) {
            // the sample's points in the layout's Hilbert order
            HIPCHK(launch_sample_compact(r, rk, sz, xb, wb, s));
            bkm_points ps = *pts;
            ps.n = sz;
            for (int j = 0; j < r.d; ++j) ps.coords[j] = xb[j];
            ps.weights = wb;
            bkm_info si;
            rc = run_core(&ps, q, cbuf, (sample_rounds || influence_init) ? ibuf : nullptr, abuf,
                          cbuf, ibuf, nullptr, &si, s, true);
            if (rc < 0) return rc;
            sample_rounds += 1;
            sample_sweeps += si.sweeps;
        }
        cinit = cbuf;
        iinit = ibuf;
    }
    if (!cinit) HIPCHK(launch_centers_from_sorted(r, r.C, 0, s));
    HIPCHK(launch_init_run(r, cinit, iinit, p.max_iter, p.max_balance_iter, p.epsilon, dthr, s));
    HIPCHK(hipEventRecord(ev[1], s));

    // One sweep per batch: most AssignAndBalance calls balance after their
    // first sweep, and a batch of one never launches a sweep that has nothing
    // to do.  Every batch ends a call or adds a sweep to it, so the loop is
    // bounded.  One batch runs ahead: batch b+1 is enqueued before the host
    // waits for the state copied at the end of batch b, so the device never
    // idles on the host's decision; a batch enqueued after the end is a no-op.
    const bool timing = p.timing != 0;
    struct LoopRes {
        hipStream_t s;
        hipEvent_t ev[2][7] = {};
        DevState* ring = nullptr;
        ~LoopRes()
        {
            (void)hipStreamSynchronize(s);   // no copy into the ring may be left in flight
            for (auto& row : ev)
                for (auto e : row)
                    if (e) (void)hipEventDestroy(e);
        }
    } lr{s};
    lr.ring = loop_ring();
    if (!lr.ring) return fail(BKM_ENOMEM, "pinned host buffer unavailable");
    for (auto& row : lr.ev) {
        for (int i = 0; i < 6; ++i)
            if (timing) HIPCHK(hipEventCreate(&row[i]));
        HIPCHK(hipEventCreateWithFlags(&row[6], hipEventDisableTiming));
    }
    double tk[5] = {0, 0, 0, 0, 0};
    auto enqueue = [&](int64_t nb) -> int {
        hipEvent_t* ev = lr.ev[nb & 1];
        auto mark = [&](int i) -> hipError_t { return timing ? hipEventRecord(ev[i], s) : hipSuccess; };
        HIPCHK(mark(0));
        HIPCHK(launch_supercand(r, s));
        HIPCHK(launch_tilecand(r, s));
        HIPCHK(mark(1));
        HIPCHK(launch_sweep(r, s));
        HIPCHK(launch_check_bounds(r, 1, s));
        HIPCHK(mark(2));
        HIPCHK(launch_balance(r, s));
        HIPCHK(mark(3));
        HIPCHK(launch_block_boxes(r, s));
        HIPCHK(mark(4));
        HIPCHK(launch_move(r, s));
        HIPCHK(launch_check_bounds(r, 0, s));
        HIPCHK(mark(5));
        HIPCHK(hipMemcpyAsync(&lr.ring[nb & 1], r.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ev[6], s));
        return BKM_OK;
    };
    DevState h;
    int prev_rounds = 0;
    const int64_t max_batches = (int64_t)p.max_iter * (p.max_balance_iter + 1) + 8;
    if ((rc = enqueue(0))) return rc;
    for (int64_t nb = 0;; ++nb) {
        if (nb >= max_batches) return fail(BKM_EHIP, "round loop made no progress");
        if ((rc = enqueue(nb + 1))) return rc;
        HIPCHK(hipEventSynchronize(lr.ev[nb & 1][6]));
        h = lr.ring[nb & 1];
        const bool round_ended = h.rounds > prev_rounds;
        if (timing) {
            for (int i = 0; i < 5; ++i) {
                if (i >= 3 && !round_ended) continue;
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, lr.ev[nb & 1][i], lr.ev[nb & 1][i + 1]));
                tk[i] += ms;
            }
        }
        prev_rounds = h.rounds;
        if (h.done) break;
    }
    HIPCHK(launch_finish(r, assignment_out, centers_out, influence_out, block_weights_out, s));
    HIPCHK(hipEventRecord(ev[2], s));
    if ((rc = read_state(r, s, &h))) return rc;
    unsigned long long cnt[kCntWords];
    if ((rc = read_counters(r, s, cnt))) return rc;
    if (cnt[kCntInvalid])
        return fail(BKM_EINTERNAL, "%llu sweep decisions produced no valid block",
                    (unsigned long long)cnt[kCntInvalid]);
    if (cnt[kCntDebugViolated])
        return fail(BKM_EINTERNAL, "debug checks: %llu of %llu checked points violate a bound "
                    "or are not at an argmin", (unsigned long long)cnt[kCntDebugViolated],
                    (unsigned long long)cnt[kCntDebugChecked]);

    if (info) {
        fill_info(info, h, cnt);
        info->sample_rounds = sample_rounds;
        info->sample_sweeps = sample_sweeps;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) info->bootstrap_ms = ms;
        if (hipEventElapsedTime(&ms, ev[0], ev[2]) == hipSuccess) info->total_ms = ms;
        info->cand_ms = tk[0];
        info->sweep_ms = tk[1];
        info->balance_ms = tk[2];
        info->boxes_ms = tk[3];
        info->move_ms = tk[4];
    }
    return h.balanced ? BKM_OK : BKM_WUNBALANCED;
}

}  // namespace

// ------------------------------------------------------- partition stats
int check_stats_args(const bkm_points* pts, const int32_t* assignment, int32_t k, double eps,
                     const bkm_stats* out)
{
    int rc = check_points(pts);
    if (rc) return rc;
    if (k < 1) return fail(BKM_EINVAL, "k = %d < 1", k);
    if (!assignment || !out) return fail(BKM_EINVAL, "assignment/out is NULL");
    if (!(eps >= 0.0)) return fail(BKM_EINVAL, "epsilon must be >= 0");
    return BKM_OK;
}

// Device workspace of the statistics: state, reduction buffer (bounding-box
// and objective partials of at most 1024 blocks), centers, fixed-point sums,
// the six results and, with target sizes, per-block targets and limits.
size_t stats_workspace(int k, int d, bool targets)
{
    Sizes z;
    z.add<DevState>(1);
    z.add<double>(std::max<int64_t>(32768, k));
    z.add<double>((size_t)k * d);
    z.add<long long>((size_t)k * kAcc);
    z.add<double>(8);
    if (targets) {
        z.add<double>((size_t)k);
        z.add<double>((size_t)k);
        z.add<double>((size_t)k + 1);
    }
    return z.total;
}

// The statistics on a workspace of stats_workspace() bytes at `ws`.  With
// `noalloc` nothing is allocated: the state is cleared by a fill kernel and
// read back into a stack copy (no pinned staging buffer).
int stats_core(const bkm_points* pts, const int32_t* assignment, int32_t k, double epsilon,
               const double* target_sizes, double* block_weights_out, double* centers_out,
               bkm_stats* out, hipStream_t s, char* ws, bool noalloc)
{
    RunDev r;
    plan(r, pts, k, 1024, 16, BKM_PREC_F64, 0, 0.0);
    Arena a;   // carves only: base is handed back before it would be freed
    a.base = ws;
    r.st = a.take<DevState>(1);
    r.red = a.take<double>(std::max<int64_t>(32768, k));
    r.C = a.take<double>((size_t)k * r.d);
    r.acc = a.take<long long>((size_t)k * kAcc);
    double* out6 = a.take<double>(8);
    if (target_sizes) {
        r.tsz = target_sizes;
        r.tT = a.take<double>((size_t)k);
        r.tL = a.take<double>((size_t)k);
        r.tpre = a.take<double>((size_t)k + 1);
    }
    a.base = nullptr;
    static_assert(sizeof(DevState) % 4 == 0, "state is cleared as 32-bit words");
    HIPCHK(launch_fill_i32((int32_t*)r.st, (int64_t)(sizeof(DevState) / 4), 0, s));
    HIPCHK(launch_fill_i32((int32_t*)r.acc, (int64_t)k * kAcc * 2, 0, s));
    HIPCHK(launch_bbox(r, 16, s));
    if (r.tsz) HIPCHK(launch_target_prep(r, epsilon, s));
    HIPCHK(launch_stats(r, assignment, epsilon, block_weights_out, centers_out, out6, s));
    double h6[8];
    HIPCHK(hipMemcpyAsync(h6, out6, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    DevState h;
    if (noalloc) {
        HIPCHK(hipMemcpyAsync(&h, r.st, sizeof(DevState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } else {
        HIPCHK(hipStreamSynchronize(s));
        int rc = read_state(r, s, &h);
        if (rc) return rc;
    }
    if (h.bad_data & 4)
        return fail(BKM_EINVAL, "target_sizes must be finite and > 0, with a finite sum");
    if (h.bad_data & 2) return fail(BKM_EINVAL, "assignment outside [0, k)");
    if (h.bad_data & 1) return fail(BKM_EDATA, "non-finite coordinate or bad weight");
    out->imbalance = h6[0];
    out->objective = h6[1];
    out->l_max = h6[2];
    out->empty_blocks = (int32_t)h6[3];
    out->overloaded_blocks = (int32_t)h6[4];
    return BKM_OK;
}

extern "C" {

void bkm_default_params(bkm_params* p, int32_t k)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->k = k;
    p->max_iter = 50;
    p->max_balance_iter = 20;
    p->hilbert_order = 16;
    p->precision = BKM_PREC_F32_RECHECK;
    p->use_bounds = 1;
    p->tile_points = 0;
    p->super_tiles = 0;
    p->timing = 0;
    p->sample_init = 0;
    p->sample_start = 0;
    p->seed = 0;
    p->sample_keys = nullptr;
    p->target_sizes = nullptr;
    p->erosion = 1;
    p->epsilon = 0.03;
    p->delta_threshold = -1.0;
    p->recheck_rel_gap = 1e-5;
}

int bkm_knn(const bkm_points* pts, int32_t knn, int32_t* nbr_out, int32_t* order_out,
            bkm_knn_info* info, void* stream)
{
    g_err.clear();
    int rc = check_points(pts);
    if (rc) return rc;
    if (knn < 1 || knn > 16) return fail(BKM_EINVAL, "knn = %d outside [1, 16]", knn);
    if (knn > pts->n - 1) return fail(BKM_EINVAL, "knn = %d needs at least knn + 1 points", knn);
    if (!nbr_out) return fail(BKM_EINVAL, "nbr_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    // the search walks the box hierarchy of the tiled Hilbert layout
    RunDev r;
    plan(r, pts, 1, 256, 16, BKM_PREC_F64, 0, 0.0);
    Arena a;
    if ((rc = alloc_run(r, a, s, true))) return rc;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    struct EvFree { hipEvent_t* e; ~EvFree() { for (int i = 0; i < 3; ++i) if (e[i]) (void)hipEventDestroy(e[i]); } } evf{ev};
    if (info)
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    if (info) HIPCHK(hipEventRecord(ev[0], s));
    if ((rc = bootstrap(r, 16, s, true))) return rc;
    // the search reads FP64 coordinates: an FP32 layout is widened first
    KnnPts P{};
    Arena wide;
    if (r.in_f32) {
        wide.s = s;
        const size_t bytes = (size_t)r.npad * r.d * sizeof(double);
        hipError_t e = hipMallocAsync((void**)&wide.base, bytes, s);
        if (e != hipSuccess) {
            wide.base = nullptr;
            return fail(e == hipErrorOutOfMemory ? BKM_ENOMEM : BKM_EHIP,
                        "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
        }
        double* x = reinterpret_cast<double*>(wide.base);
        HIPCHK(launch_knn_widen(r, x, s));
        for (int j = 0; j < r.d; ++j) P.x[j] = x + (size_t)j * r.npad;
    } else {
        for (int j = 0; j < r.d; ++j) P.x[j] = r.xs64[j];
    }
    // boxes of the groups' 8-point parts
    Arena parts;
    {
        parts.s = s;
        const size_t bytes = (size_t)r.ngroups * kKnnParts * 2 * r.d * sizeof(double);
        hipError_t e = hipMallocAsync((void**)&parts.base, bytes, s);
        if (e != hipSuccess) {
            parts.base = nullptr;
            return fail(e == hipErrorOutOfMemory ? BKM_ENOMEM : BKM_EHIP,
                        "hipMallocAsync(%zu bytes): %s", bytes, hipGetErrorString(e));
        }
        double* pb = reinterpret_cast<double*>(parts.base);
        HIPCHK(launch_knn_partbox(r, P, pb, s));
        P.pbox = pb;
    }
    unsigned long long* visits = reinterpret_cast<unsigned long long*>(r.red);
    HIPCHK(hipMemsetAsync(visits, 0, sizeof(unsigned long long), s));
    if (info) HIPCHK(hipEventRecord(ev[1], s));
    HIPCHK(launch_knn(r, P, knn, nbr_out, visits, s));
    if (info) HIPCHK(hipEventRecord(ev[2], s));
    if (order_out)
        HIPCHK(hipMemcpyAsync(order_out, r.sperm, (size_t)r.n * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
    unsigned long long hv = 0;
    HIPCHK(hipMemcpyAsync(&hv, visits, sizeof(hv), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (info) {
        float t01 = 0.f, t12 = 0.f;
        HIPCHK(hipEventElapsedTime(&t01, ev[0], ev[1]));
        HIPCHK(hipEventElapsedTime(&t12, ev[1], ev[2]));
        info->group_visits = (int64_t)(hv / kKnnParts);   // counted in 8-point parts
        info->layout_ms = t01;
        info->search_ms = t12;
    }
    return BKM_OK;
}

int bkm_knn_graph(int64_t n, int32_t knn, const int32_t* nbr, const int32_t* order,
                  int64_t* row_ptr_out, int32_t* col_out, int64_t* nnz_out, void* stream)
{
    g_err.clear();
    if (n < 2 || n > INT32_MAX) return fail(BKM_EINVAL, "n = %lld outside [2, 2^31-1]", (long long)n);
    if (knn < 1 || knn > n - 1) return fail(BKM_EINVAL, "knn = %d outside [1, n-1]", knn);
    if (!nbr || !row_ptr_out || !col_out) return fail(BKM_EINVAL, "nbr/row_ptr_out/col_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    Sizes z;
    z.add<int32_t>((size_t)n);
    z.add<int32_t>((size_t)n);
    z.add<int64_t>((size_t)scan_parts(n));
    z.add<int>(1);
    const size_t nmiss = (size_t)((n * knn + kWave - 1) / kWave);
    z.add<unsigned long long>(nmiss);
    Arena a;
    a.s = s;
    HIPCHK(hipMallocAsync((void**)&a.base, z.total, s));
    a.cap = z.total;
    int32_t* extra = a.take<int32_t>((size_t)n);
    int32_t* cursor = a.take<int32_t>((size_t)n);
    int64_t* part = a.take<int64_t>((size_t)scan_parts(n));
    int* bad = a.take<int>(1);
    unsigned long long* miss = a.take<unsigned long long>(nmiss);   // written whole by the count
    HIPCHK(hipMemsetAsync(extra, 0, (size_t)n * sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(cursor, 0, (size_t)n * sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
    int hb = 0;
    if (order) {
        // cursor (zero) serves as the permutation check's marks and is zero again after it
        HIPCHK(launch_order_check(n, order, cursor, bad, s));
        HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hb) return fail(BKM_EINVAL, "order is not a permutation of 0..n-1");
    }
    HIPCHK(launch_sym_count(n, knn, nbr, order, extra, miss, bad, s));
    HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb) return fail(BKM_EINVAL, "neighbour entry outside [0, n) or pointing to its own row");
    HIPCHK(launch_sym_rows(n, knn, extra, part, row_ptr_out, s));
    HIPCHK(launch_sym_fill(n, knn, nbr, order, miss, row_ptr_out, cursor, col_out, s));
    int64_t nnz = 0;
    HIPCHK(hipMemcpyAsync(&nnz, row_ptr_out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nnz_out) *nnz_out = nnz;
    return BKM_OK;
}

int bkm_graph_metrics(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                      const int32_t* assignment, int32_t k, int64_t* comm_out,
                      int32_t* diameter_out, int32_t* diameter_ub_out, bkm_graph_stats* out,
                      void* stream)
{
    g_err.clear();
    if (n < 1 || n > INT32_MAX) return fail(BKM_EINVAL, "n = %lld outside [1, 2^31-1]", (long long)n);
    if (nnz < 0) return fail(BKM_EINVAL, "nnz < 0");
    if (k < 1) return fail(BKM_EINVAL, "k = %d < 1", k);
    if (!row_ptr || (!col && nnz > 0) || !assignment || !out)
        return fail(BKM_EINVAL, "row_ptr/col/assignment/out is NULL");
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    constexpr int kBlockInts = 12;  // per-block int32 arrays of GraphDev
    Sizes z;
    z.add<int64_t>((size_t)k);
    for (int i = 0; i < kBlockInts; ++i) z.add<int32_t>((size_t)k);
    z.add<int32_t>((size_t)k + 1);
    z.add<long long>(4);
    z.add<int>(16);
    z.add<double>(8);
    for (int i = 0; i < 7; ++i) z.add<int32_t>((size_t)n);
    z.add<int2>((size_t)n);
    for (int i = 0; i < 3; ++i) z.add<unsigned long long>((size_t)n);
    z.add<int64_t>((size_t)n + 1);
    z.add<int32_t>((size_t)std::max<int64_t>(nnz, 1));
    z.add<int64_t>((size_t)scan_parts(n));
    Arena a;
    a.s = s;
    HIPCHK(hipMallocAsync((void**)&a.base, z.total, s));
    a.cap = z.total;
    GraphDev g;
    g.comm = a.take<int64_t>((size_t)k);
    int32_t* bi[kBlockInts];
    for (int i = 0; i < kBlockInts; ++i) bi[i] = a.take<int32_t>((size_t)k);
    g.size = bi[0];
    g.seed = bi[1];
    g.conn = bi[2];
    g.fill = bi[3];
    g.ecc1 = bi[4];
    g.lval = bi[5];
    g.fi = bi[6];
    g.lb = bi[7];
    g.ub = bi[8];
    g.far1 = bi[9];
    g.nlev = bi[10];
    g.clist = bi[11];
    g.moff = a.take<int32_t>((size_t)k + 1);
    long long* sc = a.take<long long>(4);
    g.cut2 = sc;
    g.sums = sc + 1;
    int* ints = a.take<int>(16);
    g.bad = ints;
    int32_t* nlevels = ints + 1;   // most levels of one block's searches
    g.ccount = ints + 2;
    double* summary = a.take<double>(8);
    g.mem = a.take<int32_t>((size_t)n);
    int32_t* dist = a.take<int32_t>((size_t)n);
    int32_t* du = a.take<int32_t>((size_t)n);
    int32_t* qa = a.take<int32_t>((size_t)n);
    int32_t* qb = a.take<int32_t>((size_t)n);
    int32_t* fr = a.take<int32_t>((size_t)n);   // the blocks' fringes, at their list offsets
    unsigned long long* seen = a.take<unsigned long long>((size_t)n);
    unsigned long long* arr0 = a.take<unsigned long long>((size_t)n);
    unsigned long long* arr1 = a.take<unsigned long long>((size_t)n);
    g.ldeg = a.take<int32_t>((size_t)n);
    g.al = a.take<int2>((size_t)n);
    g.lrp = a.take<int64_t>((size_t)n + 1);
    g.lcol = a.take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
    int64_t* part = a.take<int64_t>((size_t)scan_parts(n));
    HIPCHK(hipMemsetAsync(g.comm, 0, (size_t)k * sizeof(int64_t), s));
    HIPCHK(hipMemsetAsync(g.size, 0, (size_t)k * sizeof(int32_t), s));
    HIPCHK(hipMemsetAsync(g.conn, 0, (size_t)k * sizeof(int32_t), s));
    HIPCHK(launch_fill_i32(g.seed, k, INT32_MAX, s));
    HIPCHK(hipMemsetAsync(sc, 0, 4 * sizeof(long long), s));
    HIPCHK(hipMemsetAsync(ints, 0, 16 * sizeof(int), s));
    HIPCHK(launch_gm_vertex(n, nnz, row_ptr, col, assignment, k, g, s));
    int hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, g.bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb) return fail(BKM_EINVAL, "assignment outside [0, k), or row_ptr/col outside the graph");
    // the diameter bounds: the block lists, the first search of every block
    // (on the input graph), the relabelled subgraphs of the connected blocks
    // (fr holds the local degrees until the searches), then the rest of their
    // searches, workgroups sized to their count
    HIPCHK(launch_block_lists(n, assignment, k, g, s));
    HIPCHK(launch_diam_first(row_ptr, col, assignment, k, g, dist, qa, qb, nlevels, s));
    HIPCHK(launch_local_rows(n, row_ptr, col, assignment, g, fr, part, s));
    int nconn = 0;
    HIPCHK(hipMemcpyAsync(&nconn, g.ccount, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (nconn < 0 || nconn > k)
        return fail(BKM_EHIP, "connected block count %d outside [0, %d]", nconn, k);
    // with more connected blocks than CUs, the shortest first (by the levels
    // of their first search): a CU's second workgroup is then one of the
    // longest, next to one of the shortest
    int dev = 0, ncu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (nconn > ncu) {
        std::vector<int32_t> cl((size_t)nconn), lv((size_t)k);
        HIPCHK(hipMemcpyAsync(cl.data(), g.clist, (size_t)nconn * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(lv.data(), g.nlev, (size_t)k * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int32_t b : cl)
            if (b < 0 || b >= k) return fail(BKM_EHIP, "connected block %d outside [0, %d)", b, k);
        std::sort(cl.begin(), cl.end(), [&](int32_t x, int32_t y) {
            return lv[x] < lv[y] || (lv[x] == lv[y] && x < y);
        });
        HIPCHK(hipMemcpyAsync(g.clist, cl.data(), (size_t)nconn * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(launch_diam_rest(nconn, g, dist, du, qa, qb, fr, seen, arr0, arr1, nlevels, s));
    int levels = 0;
    HIPCHK(hipMemcpyAsync(&levels, nlevels, sizeof(levels), hipMemcpyDeviceToHost, s));
    HIPCHK(launch_gm_final(k, g, diameter_out, diameter_ub_out, comm_out, summary, s));
    double hs[8];
    long long hl[4];
    HIPCHK(hipMemcpyAsync(hs, summary, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hl, sc, sizeof(hl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof(*out));
    out->edge_cut = hl[0] / 2;
    out->max_comm = hl[1];
    out->total_comm = hl[2];
    out->disconnected_blocks = (int32_t)hl[3];
    out->max_diameter = (int32_t)hs[3];
    const double inv = hs[4], counted = hs[5];
    out->harmonic_diameter = counted == 0.0 ? 0.0 : (inv == 0.0 ? INFINITY : counted / inv);
    out->bfs_levels = levels;
    out->exact_blocks = (int32_t)hs[6];
    return BKM_OK;
}

const char* bkm_last_error(void) { return g_err.c_str(); }

int bkm_autotune(const bkm_points* pts, const bkm_params* prm, int32_t force,
                 bkm_tune_result* out, void* stream)
{
    g_err.clear();
    int rc = check_run(pts, prm);
    if (rc) return rc;
    if (!out) return fail(BKM_EINVAL, "out is NULL");
    keep_pool_memory();
    int T = 0, ST = 0;
    rc = tuned_tiles(pts, *prm, (hipStream_t)stream, &T, &ST, out, force != 0);
    return rc < 0 ? rc : BKM_OK;
}

void bkm_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

int bkm_init_centers_sfc(const bkm_points* pts, int32_t k, int32_t hilbert_order,
                         double* centers_out, int32_t* perm_out, uint64_t* keys_out,
                         void* stream)
{
    g_err.clear();
    int rc = check_points(pts);
    if (rc) return rc;
    if (k < 1 || k > pts->n) return fail(BKM_EINVAL, "k = %d outside [1, n]", k);
    if ((rc = check_order(pts->d, hilbert_order))) return rc;
    if (!centers_out) return fail(BKM_EINVAL, "centers_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    RunDev r;
    plan(r, pts, k, 1024, 16, BKM_PREC_F64, 0, 0.0);
    Arena a;
    if ((rc = alloc_run(r, a, s, false))) return rc;
    HIPCHK(launch_bbox(r, hilbert_order, s));
    DevState h;
    if ((rc = read_state(r, s, &h))) return rc;
    if (h.bad_data) return fail(BKM_EDATA, "non-finite coordinate");
    HIPCHK(launch_keys(r, hilbert_order, r.sperm, s));
    if (keys_out)
        HIPCHK(hipMemcpyAsync(keys_out, r.keys, r.n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(radix_sort_pairs(r, r.keys, r.sperm, r.d * hilbert_order, s));
    HIPCHK(launch_permute(r, s));
    HIPCHK(launch_centers_from_sorted(r, centers_out, 1, s));
    if (perm_out)
        HIPCHK(hipMemcpyAsync(perm_out, r.sperm, r.n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return BKM_OK;
}

int bkm_balanced_kmeans(const bkm_points* pts, const bkm_params* prm, const double* centers_init,
                        int32_t* assignment_out, double* centers_out, double* influence_out,
                        double* block_weights_out, bkm_info* info, void* stream)
{
    g_err.clear();
    int rc = check_run(pts, prm);
    if (rc) return rc;
    if (!assignment_out || !centers_out) return fail(BKM_EINVAL, "assignment_out/centers_out is NULL");
    keep_pool_memory();
    return run_core(pts, *prm, centers_init, nullptr, assignment_out, centers_out, influence_out,
                    block_weights_out, info, (hipStream_t)stream);
}

int bkm_assign_sweeps(const bkm_points* pts, int32_t k, int32_t steps, const double* centers,
                      const double* influence, int32_t precision, int32_t use_bounds,
                      int32_t tile_points, int32_t* assignment_out, double* block_weights_out,
                      bkm_info* info, void* stream)
{
    g_err.clear();
    int rc = check_points(pts);
    if (rc) return rc;
    if (k < 1 || k > pts->n) return fail(BKM_EINVAL, "k = %d outside [1, n]", k);
    if (steps < 1) return fail(BKM_EINVAL, "steps must be >= 1");
    if (!centers || !influence || !assignment_out)
        return fail(BKM_EINVAL, "centers/influence/assignment_out is NULL");
    if (precision != BKM_PREC_F64 && precision != BKM_PREC_F32_RECHECK)
        return fail(BKM_EINVAL, "precision %d unknown", precision);
    if (!check_tile(tile_points)) return fail(BKM_EINVAL, "tile_points %d not 0/256/512/1024", tile_points);
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    RunDev r;
    plan(r, pts, k, tile_points ? tile_points : 1024, 16, precision, use_bounds ? 1 : 0, 1e-5);
    Arena a;
    if ((rc = alloc_run(r, a, s, true))) return rc;
    if ((rc = bootstrap(r, 16, s, true))) return rc;
    HIPCHK(launch_init_run(r, nullptr, nullptr, 1, 1, 0.0, -1.0, s));
    for (int t = 0; t < steps; ++t) {
        HIPCHK(launch_set_step(r, centers + (int64_t)t * k * r.d, influence + (int64_t)t * k,
                               t == 0, s));
        HIPCHK(launch_supercand(r, s));
        HIPCHK(launch_tilecand(r, s));
        HIPCHK(launch_sweep(r, s));
        HIPCHK(launch_finish(r, assignment_out + (int64_t)t * r.n, nullptr, nullptr,
                             block_weights_out ? block_weights_out + (int64_t)t * k : nullptr, s));
    }
    unsigned long long cnt[kCntWords];
    if ((rc = read_counters(r, s, cnt))) return rc;
    if (cnt[kCntInvalid])
        return fail(BKM_EINTERNAL, "%llu sweep decisions produced no valid block",
                    (unsigned long long)cnt[kCntInvalid]);
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->sweeps = steps;
        info->evaluated = (int64_t)cnt[kCntEvaluated];
        info->skipped = (int64_t)cnt[kCntSkipped];
        info->rechecked = (int64_t)cnt[kCntRechecked];
        info->changed = (int64_t)cnt[kCntChanged];
        info->candidate_evals = (int64_t)cnt[kCntCandEvals];
        info->overflow_tiles = (int64_t)cnt[kCntOverflow];
    }
    return BKM_OK;
}

int bkm_partition_stats(const bkm_points* pts, const int32_t* assignment, int32_t k,
                        double epsilon, const double* target_sizes, double* block_weights_out,
                        double* centers_out, bkm_stats* out, void* stream)
{
    g_err.clear();
    int rc = check_stats_args(pts, assignment, k, epsilon, out);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    const size_t bytes = stats_workspace(k, pts->d, target_sizes != nullptr);
    Arena a;
    a.s = s;
    HIPCHK(hipMallocAsync((void**)&a.base, bytes, s));
    return stats_core(pts, assignment, k, epsilon, target_sizes, block_weights_out, centers_out,
                      out, s, a.base, false);
}

int bkm_partition_stats_noalloc(const bkm_points* pts, const int32_t* assignment, int32_t k,
                                double epsilon, const double* target_sizes,
                                double* block_weights_out, double* centers_out, bkm_stats* out,
                                void* stream)
{
    g_err.clear();
    int rc = check_stats_args(pts, assignment, k, epsilon, out);
    if (rc) return rc;
    if (k > BKM_NOALLOC_MAX_K)
        return fail(BKM_EINVAL, "k = %d above the no-allocation limit %d", k, BKM_NOALLOC_MAX_K);
    const size_t bytes = stats_workspace(k, pts->d, target_sizes != nullptr);
    if (bytes > sizeof(scratch))
        return fail(BKM_EINVAL, "workspace of %zu bytes exceeds the static %zu", bytes,
                    sizeof(scratch));
    char* ws = nullptr;
    if ((rc = scratch_address(&ws))) return rc;
    return stats_core(pts, assignment, k, epsilon, target_sizes, block_weights_out, centers_out,
                      out, (hipStream_t)stream, ws, true);
}

int bkm_balanced_kmeans_batched(const bkm_points* pts, const bkm_params* prm, int32_t count,
                                int32_t* const* assignment_out, double* const* centers_out,
                                bkm_info* info, void* stream)
{
    g_err.clear();
    if (count < 1) return fail(BKM_EINVAL, "count = %d must be >= 1", count);
    if (!pts || !prm || !assignment_out || !centers_out)
        return fail(BKM_EINVAL, "points/params/assignment_out/centers_out array is NULL");
    for (int i = 0; i < count; ++i) {
        int rc = check_run(&pts[i], &prm[i]);
        if (!rc && (!assignment_out[i] || !centers_out[i]))
            rc = fail(BKM_EINVAL, "assignment_out/centers_out is NULL");
        if (!rc && prm[i].sample_init)
            rc = fail(BKM_EINVAL, "sample_init is not supported by the batched call");
        if (rc) {
            g_err = "instance " + std::to_string(i) + ": " + g_err;
            return rc;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    keep_pool_memory();
    BatchRes res;
    hipEvent_t t0, t1, t2;
    for (hipEvent_t* e : {&t0, &t1, &t2}) {
        HIPCHK(hipEventCreate(e));
        res.events.push_back(*e);
    }
    HIPCHK(hipEventRecord(t0, s));

    // one workspace for all instances; their run states side by side, so a
    // single copy reads them all
    std::vector<RunDev> rs(count);
    Sizes z;
    z.add<DevState>(count);
    for (int i = 0; i < count; ++i) {
        const bkm_params& p = prm[i];
        int T = p.tile_points > 0 ? p.tile_points : auto_tile(pts[i].n, p.k);
        int ST = p.super_tiles ? p.super_tiles : 16;
        if (p.tile_points == 0) {
            const int rc = tuned_tiles(&pts[i], p, s, &T, &ST, nullptr);
            if (rc < 0) return rc;
        }
        plan(rs[i], &pts[i], p.k, T, ST, p.precision, p.use_bounds ? 1 : 0, p.recheck_rel_gap);
        rs[i].tsz = p.target_sizes;
        rs[i].erosion = p.erosion;
        z.total += layout(rs[i], nullptr, true);
    }
    Arena a;
    a.s = s;
    // on an early return, the worker streams finish before the workspace goes
    struct SyncWorkers {
        std::vector<hipStream_t>& v;
        ~SyncWorkers() { for (auto q : v) (void)hipStreamSynchronize(q); }
    } sync_workers{res.streams};
    {
        hipError_t e = hipMallocAsync((void**)&a.base, z.total, s);
        if (e != hipSuccess) {
            a.base = nullptr;
            return fail(e == hipErrorOutOfMemory ? BKM_ENOMEM : BKM_EHIP,
                        "hipMallocAsync(%zu bytes): %s", z.total, hipGetErrorString(e));
        }
        a.cap = z.total;
    }
    DevState* states = a.take<DevState>(count);
    for (int i = 0; i < count; ++i) {
        layout(rs[i], &a, true);
        rs[i].st = states + i;
    }
    HIPCHK(hipMemsetAsync(states, 0, (size_t)count * sizeof(DevState), s));
    HIPCHK(hipHostMalloc((void**)&res.hstates, (size_t)count * sizeof(DevState), hipHostMallocDefault));
    auto read_all = [&]() -> int {
        HIPCHK(hipMemcpyAsync(res.hstates, states, (size_t)count * sizeof(DevState),
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return BKM_OK;
    };

    // bootstrap: instances spread over worker streams, in three phases split
    // by the two host reads (data checks, padded layout sizes)
    const int W = std::min(count, 8);
    for (int w = 0; w < W; ++w) {
        hipStream_t q;
        HIPCHK(hipStreamCreateWithFlags(&q, hipStreamNonBlocking));
        res.streams.push_back(q);
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        res.events.push_back(e);
    }
    hipEvent_t efork;
    HIPCHK(hipEventCreateWithFlags(&efork, hipEventDisableTiming));
    res.events.push_back(efork);
    auto fork = [&]() -> int {
        HIPCHK(hipEventRecord(efork, s));
        for (auto q : res.streams) HIPCHK(hipStreamWaitEvent(q, efork, 0));
        return BKM_OK;
    };
    auto join = [&]() -> int {
        for (int w = 0; w < W; ++w) {
            hipEvent_t e = res.events[3 + w];
            HIPCHK(hipEventRecord(e, res.streams[w]));
            HIPCHK(hipStreamWaitEvent(s, e, 0));
        }
        return BKM_OK;
    };
    int rc;
    if ((rc = fork())) return rc;
    for (int i = 0; i < count; ++i) {
        HIPCHK(launch_bbox(rs[i], prm[i].hilbert_order, res.streams[i % W]));
        if (rs[i].tsz) HIPCHK(launch_target_prep(rs[i], prm[i].epsilon, res.streams[i % W]));
    }
    if ((rc = join()) || (rc = read_all())) return rc;
    for (int i = 0; i < count; ++i)
        if (res.hstates[i].bad_data & 4)
            return fail(BKM_EINVAL, "instance %d: target_sizes must be finite and > 0, with a finite sum", i);
    for (int i = 0; i < count; ++i)
        if (res.hstates[i].bad_data)
            return fail(BKM_EDATA, "instance %d: %s", i,
                        rs[i].weighted ? "non-finite coordinate or weight <= 0 / non-finite"
                                       : "non-finite coordinate");
    if ((rc = fork())) return rc;
    for (int i = 0; i < count; ++i) {
        RunDev& r = rs[i];
        hipStream_t q = res.streams[i % W];
        HIPCHK(launch_keys(r, prm[i].hilbert_order, r.sperm, q));
        HIPCHK(radix_sort_pairs(r, r.keys, r.sperm, r.d * prm[i].hilbert_order, q));
        HIPCHK(launch_permute(r, q));
        HIPCHK(launch_jump_plan(r, q));
    }
    if ((rc = join()) || (rc = read_all())) return rc;
    for (int i = 0; i < count; ++i) {
        const int64_t np = res.hstates[i].npad;
        if (np < rs[i].n || np > rs[i].npad_cap)
            return fail(BKM_EHIP, "instance %d: padded layout of %lld points outside [n, %lld]", i,
                        (long long)np, (long long)rs[i].npad_cap);
        set_layout_size(rs[i], np);
    }
    if ((rc = fork())) return rc;
    for (int i = 0; i < count; ++i) {
        const RunDev& r = rs[i];
        const bkm_params& p = prm[i];
        hipStream_t q = res.streams[i % W];
        HIPCHK(launch_place(r, q));
        HIPCHK(launch_tile_prep(r, q));
        HIPCHK(launch_centers_from_sorted(r, r.C, 0, q));
        HIPCHK(launch_init_run(r, nullptr, nullptr, p.max_iter, p.max_balance_iter, p.epsilon,
                               p.delta_threshold, q));
    }
    if ((rc = join())) return rc;
    HIPCHK(hipEventRecord(t1, s));

    // Classes of the still active instances that share kernels, with the
    // block maps of their per-sweep launches, and the round loop captured in
    // a graph over them: kGraphBatches batches (every class: candidates,
    // sweep, balance, round end, move), replayed until every instance is
    // done.  An instance that is done turns its kernels into no-ops; when the
    // active set has shrunk by a fifth, the maps and the graph are rebuilt
    // without the finished instances, so their blocks stop being launched.
    // The loop runs on a worker stream (capture needs a stream of its own),
    // joined to the caller's stream before and after.
    hipStream_t ls = res.streams[0];
    HIPCHK(hipEventRecord(efork, s));
    HIPCHK(hipStreamWaitEvent(ls, efork, 0));
    constexpr int kGraphBatches = 4;
    std::vector<MultiSet> ms;
    Arena a2;
    a2.s = ls;
    {
        // room for the maps of all instances; rebuilds reuse it from the start
        Sizes z2;
        z2.add<RunDev>(count);
        for (int i = 0; i < count; ++i) {
            const RunDev& r = rs[i];
            z2.add<int2>(r.nhyper);
            z2.add<int2>(r.nsuper);
            z2.add<int2>((r.ntiles + kBlock / kWave - 1) / (kBlock / kWave));
            z2.add<int2>(r.ntiles);
            z2.add<int2>((r.ngroups + kPassGroupsHost - 1) / kPassGroupsHost);
        }
        z2.add<int2>(count);
        z2.total += 64 * 7 * 256;  // per-class rounding (at most 24 classes of 7 arrays)
        HIPCHK(hipMallocAsync((void**)&a2.base, z2.total, ls));
        a2.cap = z2.total;
    }
    std::vector<std::vector<RunDev>> hrs;
    std::vector<std::vector<int2>> hmap;
    auto build = [&](const std::vector<int>& act) -> int {
        ms.clear();
        std::vector<std::vector<int>> cls;
        for (int i : act) {
            const RunDev& r = rs[i];
            size_t c = 0;
            for (; c < ms.size(); ++c)
                if (ms[c].d == r.d && ms[c].precision == r.precision && ms[c].ppt == r.ppt &&
                    ms[c].weighted == r.weighted)
                    break;
            if (c == ms.size()) {
                MultiSet m{};
                m.d = r.d;
                m.precision = r.precision;
                m.ppt = r.ppt;
                m.weighted = r.weighted;
                ms.push_back(m);
                cls.emplace_back();
            }
            cls[c].push_back(i);
        }
        hrs.assign(ms.size(), {});
        hmap.assign(ms.size() * 6, {});
        a2.off = 0;
        for (size_t c = 0; c < ms.size(); ++c) {
            MultiSet& m = ms[c];
            m.ninst = (int)cls[c].size();
            for (int j = 0; j < m.ninst; ++j) {
                const RunDev& r = rs[cls[c][j]];
                hrs[c].push_back(r);
                const int nq = (r.ntiles + kBlock / kWave - 1) / (kBlock / kWave);
                const int npass = (r.ngroups + kPassGroupsHost - 1) / kPassGroupsHost;
                for (int b = 0; b < r.nsuper; ++b) hmap[c * 6 + 0].push_back(make_int2(j, b));
                for (int b = 0; b < nq; ++b) hmap[c * 6 + 1].push_back(make_int2(j, b));
                for (int b = 0; b < r.ntiles; ++b) hmap[c * 6 + 2].push_back(make_int2(j, b));
                for (int b = 0; b < npass; ++b) hmap[c * 6 + 3].push_back(make_int2(j, b));
                hmap[c * 6 + 4].push_back(make_int2(j, 0));
                for (int b = 0; b < r.nhyper; ++b) hmap[c * 6 + 5].push_back(make_int2(j, b));
            }
            m.nb_super = (int)hmap[c * 6 + 0].size();
            m.nb_quad = (int)hmap[c * 6 + 1].size();
            m.nb_tile = (int)hmap[c * 6 + 2].size();
            m.nb_pass = (int)hmap[c * 6 + 3].size();
            m.nb_hyper = (int)hmap[c * 6 + 5].size();
            RunDev* drs = a2.take<RunDev>(m.ninst);
            if (a2.off > a2.cap) return fail(BKM_EHIP, "block maps exceed their workspace");
            HIPCHK(hipMemcpyAsync(drs, hrs[c].data(), m.ninst * sizeof(RunDev), hipMemcpyHostToDevice, ls));
            m.rs = drs;
            const int2** dst[6] = {&m.map_super, &m.map_quad, &m.map_tile, &m.map_pass, &m.map_inst,
                                   &m.map_hyper};
            for (int t = 0; t < 6; ++t) {
                const std::vector<int2>& v = hmap[c * 6 + t];
                int2* d = a2.take<int2>(v.size());
                if (a2.off > a2.cap) return fail(BKM_EHIP, "block maps exceed their workspace");
                if (!v.empty())
                    HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, ls));
                *dst[t] = d;
            }
        }
        HIPCHK(hipStreamSynchronize(ls));
        return BKM_OK;
    };
    auto enqueue = [&]() -> int {
        for (int g = 0; g < kGraphBatches; ++g)
            for (const MultiSet& m : ms) {
                HIPCHK(launch_sweep_multi(m, ls));
                HIPCHK(launch_update_multi(m, ls));
            }
        return BKM_OK;
    };
    bool use_graph = true;
    auto capture = [&]() -> int {
        if (res.exec) (void)hipGraphExecDestroy(res.exec);
        if (res.graph) (void)hipGraphDestroy(res.graph);
        res.exec = nullptr;
        res.graph = nullptr;
        use_graph = hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (!use_graph) return BKM_OK;
        const int erc = enqueue();
        const hipError_t e = hipStreamEndCapture(ls, &res.graph);
        if (erc) return erc;
        HIPCHK(e);
        HIPCHK(hipGraphInstantiate(&res.exec, res.graph, nullptr, nullptr, 0));
        return BKM_OK;
    };
    std::vector<int> act(count);
    for (int i = 0; i < count; ++i) act[i] = i;
    if ((rc = build(act)) || (rc = capture())) return rc;
    size_t built_for = act.size();
    int64_t max_batches = 0;
    for (int i = 0; i < count; ++i)
        max_batches = std::max<int64_t>(max_batches,
                                        (int64_t)prm[i].max_iter * (prm[i].max_balance_iter + 1) + 8);
    for (int64_t nb = 0;; nb += kGraphBatches) {
        if (nb >= max_batches + kGraphBatches) return fail(BKM_EHIP, "round loop made no progress");
        if (use_graph)
            HIPCHK(hipGraphLaunch(res.exec, ls));
        else if ((rc = enqueue()))
            return rc;
        HIPCHK(hipMemcpyAsync(res.hstates, states, (size_t)count * sizeof(DevState),
                              hipMemcpyDeviceToHost, ls));
        HIPCHK(hipStreamSynchronize(ls));
        act.clear();
        for (int i = 0; i < count; ++i)
            if (!res.hstates[i].done) act.push_back(i);
        if (act.empty()) break;
        if (act.size() * 5 <= built_for * 4) {
            if ((rc = build(act)) || (rc = capture())) return rc;
            built_for = act.size();
        }
    }
    HIPCHK(hipEventRecord(res.events[3], ls));
    HIPCHK(hipStreamWaitEvent(s, res.events[3], 0));

    for (int i = 0; i < count; ++i)
        HIPCHK(launch_finish(rs[i], assignment_out[i], centers_out[i], nullptr, nullptr, s));
    HIPCHK(hipEventRecord(t2, s));
    HIPCHK(hipHostMalloc((void**)&res.hcnt, (size_t)count * kCntSlots * kCntWords * sizeof(unsigned long long),
                         hipHostMallocDefault));
    for (int i = 0; i < count; ++i)
        HIPCHK(hipMemcpyAsync(res.hcnt + (size_t)i * kCntSlots * kCntWords, rs[i].cnt,
                              kCntSlots * kCntWords * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    if ((rc = read_all())) return rc;
    bool balanced = true;
    float boot_ms = 0.0f, tot_ms = 0.0f;
    (void)hipEventElapsedTime(&boot_ms, t0, t1);
    (void)hipEventElapsedTime(&tot_ms, t0, t2);
    for (int i = 0; i < count; ++i) {
        balanced = balanced && res.hstates[i].balanced;
        unsigned long long cnt[kCntWords];
        for (int j = 0; j < kCntWords; ++j) {
            cnt[j] = 0;
            for (int q = 0; q < kCntSlots; ++q) cnt[j] += res.hcnt[(size_t)i * kCntSlots * kCntWords + q * kCntWords + j];
        }
        if (cnt[kCntInvalid])
            return fail(BKM_EINTERNAL, "instance %d: %llu sweep decisions produced no valid block",
                        i, (unsigned long long)cnt[kCntInvalid]);
        if (!info) continue;
        fill_info(&info[i], res.hstates[i], cnt);
        info[i].bootstrap_ms = boot_ms;
        info[i].total_ms = tot_ms;
    }
    return balanced ? BKM_OK : BKM_WUNBALANCED;
}

}  // extern "C"
