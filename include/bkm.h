/*
 * bkm.h -- C ABI of libbkm, balanced k-means geometric partitioning on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: M. von Looz, C. Tzovas, H. Meyerhenke, "Balanced k-means for
 * Parallel Geometric Partitioning", arXiv:1805.01208.  Problem statement in
 * Sec. 2 and Sec. 4 (points P, block count k, imbalance eps, optional node
 * weights w: P -> R+); AssignAndBalance is Alg. 1, BalancedKMeans is Alg. 2.
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] are device (HBM) pointers on the current HIP
 *     device; [host] marks host memory.  The caller owns every buffer it
 *     passes; the library never frees or keeps them.
 *   - Points are structure-of-arrays: coords[j][i] is coordinate j of point
 *     i, each array contiguous; d is 2 or 3.
 *   - `stream` is a hipStream_t passed as void*, NULL for the default
 *     stream.  Work is ordered on that stream; every call returns after the
 *     stream has drained, so host outputs are valid on return.
 *   - Scratch memory comes from the device's default memory pool on that
 *     stream (hipMallocAsync) and is released before return.
 *   - Return value: BKM_OK (0), a negative error code (the message is in
 *     bkm_last_error()), or a positive warning.  No exception or abort ever
 *     crosses the ABI.  On an error the outputs are unspecified.
 */
#ifndef BKM_H
#define BKM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BKM_OK 0
#define BKM_EINVAL (-1)      /* bad argument: NULL pointer, d not 2/3, k < 1 or k > n,
                                eps < 0 or NaN, order out of range, ... */
#define BKM_EDATA (-2)       /* non-finite coordinate, or weight <= 0 / non-finite */
#define BKM_ENOMEM (-3)      /* device allocation failed */
#define BKM_EHIP (-4)        /* a HIP runtime call failed (message names it) */
#define BKM_EINTERNAL (-5)   /* an internal consistency check failed (a sweep decision
                                produced no valid block); outputs are not valid */
#define BKM_WUNBALANCED 1    /* outputs valid, but the last AssignAndBalance call
                                ran out of sweeps before meeting L_max */

typedef enum { BKM_F32 = 0, BKM_F64 = 1 } bkm_dtype;

/* Arithmetic of the assignment sweep.
 *   BKM_PREC_F64          every effective distance in FP64, exactly the
 *                         definition dist(p,c)/influence(c) (Sec. 4.2).
 *   BKM_PREC_F32_RECHECK  FP32 screen on tile-local coordinate offsets; a
 *                         point whose best and second-best FP32 values are
 *                         closer than max(recheck_rel_gap, the proven FP32
 *                         error) is decided again in FP64, so assignments are
 *                         the FP64 ones. */
typedef enum { BKM_PREC_F64 = 0, BKM_PREC_F32_RECHECK = 1 } bkm_precision;

typedef struct {
    int64_t n;               /* number of points, 1 <= n < 2^31 */
    int32_t d;               /* 2 or 3 */
    int32_t dtype;           /* bkm_dtype of the coordinate arrays */
    const void* coords[3];   /* [device] d arrays of n values; coords[2] unused if d == 2 */
    const double* weights;   /* [device] n node weights (> 0, finite), or NULL for unit weights */
} bkm_points;

typedef struct {
    int32_t k;                /* number of blocks, 1 <= k <= n */
    int32_t max_iter;         /* AssignAndBalance calls (Alg. 2 loop), >= 1; default 50 */
    int32_t max_balance_iter; /* sweeps per AssignAndBalance call (Alg. 1 loop), >= 1; default 20 */
    int32_t hilbert_order;    /* bits per axis of the Hilbert index: 1..31 (2D), 1..21 (3D); default 16 */
    int32_t precision;        /* bkm_precision; default BKM_PREC_F32_RECHECK */
    int32_t use_bounds;       /* 1: Hamerly upper/lower bounds skip points (Sec. 4.3); default 1 */
    int32_t tile_points;      /* points per tile of the sweep: 256, 512 or 1024; 0 = chosen
                                 by the autotuner (bkm_autotune: cached, or measured on
                                 first use); -1 = chosen from the mean number of points
                                 per block (1024 from 2048 up, 512 from 512, else 256) */
    int32_t super_tiles;      /* tiles per candidate super-tile, >= 1; 0 = the tuned value
                                 with tile_points = 0, else 16 */
    int32_t timing;           /* 1: time every kernel of the round loop with HIP events on
                                 `stream` and report the sums in bkm_info; default 0 */
    int32_t sample_init;      /* 1: random-sample initialization before the main loop (the
                                 random initialization of Sec. 4.5): rounds on
                                 the first s points of a random order, s = sample_start
                                 doubling after each round while s < n, carrying centers
                                 and influence on; each such round is one AssignAndBalance
                                 with the sample's own balance target, then one center
                                 movement with erosion; they do not count towards
                                 max_iter.  Default 0 */
    int32_t erosion;          /* 1: after each center movement that does not converge, the
                                 influence is eroded towards 1 (Sec. 4.2); 0: the influence
                                 is kept.  Default 1 */
    double epsilon;           /* imbalance eps >= 0 (may be +inf); default 0.03 */
    double delta_threshold;   /* absolute; < 0 selects 1e-5 * largest bounding-box extent
                                 (of all points, also in the sample rounds) */
    double recheck_rel_gap;   /* FP64 recheck window, relative, >= 0; default 1e-5 */
    int64_t sample_start;     /* first sample size, >= 1; 0 (default) = 100 * k: the paper
                                 starts each process with 100 of its points and uses one
                                 block per process */
    uint64_t seed;            /* random order: point i gets key splitmix64 output i of the
                                 stream seeded with `seed` (Steele, Lea, Flood 2014:
                                 z = seed + (i+1)*0x9E3779B97F4A7C15, then the mixer);
                                 ties by index.  Default 0 */
    const uint64_t* sample_keys;  /* [device] n keys in input order replacing the generated
                                     ones, or NULL */
    const double* target_sizes;   /* [device] k relative block sizes t_c (finite, > 0), or
                                     NULL for equal blocks (the footnote to the objective at
                                     the start of Sec. 4).  Block c gets target weight
                                     T_c = W*t_c/tsum (tsum summed in index order) and limit
                                     (1+eps)*ceil(n*t_c/tsum), or (1+eps)*T_c with node
                                     weights; initial center c is the sorted point
                                     floor(n*S_c/tsum) + floor(n*t_c/(2*tsum)) (S_c the sum
                                     of the sizes before c), at most n-1.  Invalid sizes
                                     give BKM_EINVAL after the bounding box is taken */
    int32_t debug_checks;     /* 0: off (default).  1: after every sweep and every center
                                 move, check sampled points against a brute-force FP64
                                 evaluation over all k centers: the stored Hamerly upper
                                 bound covers the distance to the own center, the lower
                                 bound is below the effective distance to every other
                                 center, and after a sweep the block is an argmin (ties
                                 within 1e-12); about 2^26 point-center pairs per check.
                                 2: the same on every point.  Any violation fails the call
                                 with BKM_EINTERNAL.  Ignored by the batched call. */
    int32_t pad_;
} bkm_params;

/* Counters of one bkm_balanced_kmeans call (host struct). */
typedef struct {
    int32_t rounds;           /* AssignAndBalance calls made */
    int32_t sweeps;           /* assignment sweeps made over all calls */
    int32_t balanced;         /* last call ended with every block <= its L_max */
    int32_t converged;        /* max center movement fell below delta_threshold */
    double imbalance;         /* max over blocks of weight / target - 1 of the returned
                                 assignment (target W/k, or T_c with target sizes) */
    double max_block_weight;
    double l_max;             /* (1+eps)*ceil(n/k), or (1+eps)*W/k with node weights; the
                                 largest block limit with target sizes */
    int64_t evaluated;        /* point visits that evaluated candidate centers */
    int64_t skipped;          /* point visits skipped by the bounds (Sec. 4.3) */
    int64_t rechecked;        /* evaluated visits decided again in FP64 */
    int64_t changed;          /* point visits whose block changed */
    int64_t candidate_evals;  /* (point, center) effective distances evaluated */
    int64_t overflow_tiles;   /* tile sweeps whose candidate list overflowed */
    double bootstrap_ms;      /* device time of the SFC bootstrap */
    double total_ms;          /* device time of the whole call */
    /* with params.timing: summed device time of each kernel of the round loop
       (only launches that did work are counted) */
    double cand_ms;           /* super-tile and tile candidate lists, once per sweep */
    double sweep_ms;          /* assignment sweeps */
    double balance_ms;        /* balance test + influence update, one per sweep */
    double boxes_ms;          /* block bounding boxes, one per round */
    double move_ms;           /* center move + erosion, one per round */
    int32_t sample_rounds;    /* rounds of the random-sample initialization */
    int32_t sample_sweeps;    /* sweeps made in them */
    int64_t debug_checked;    /* with params.debug_checks: points checked, over all checks */
    int64_t debug_violations; /* and those that failed (the call then fails) */
    int64_t list_builds;      /* sweeps that built the candidate lists; the others kept the
                                 lists of the last build (the influences had moved within
                                 the lists' margin) */
} bkm_info;

typedef struct {
    double imbalance;         /* max over blocks of weight / target - 1 */
    double objective;         /* sum_p w(p) * dist(p, weighted mean of its block)^2 */
    double l_max;             /* L_max; the largest block limit with target sizes */
    int32_t empty_blocks;
    int32_t overloaded_blocks; /* blocks with weight > their L_max (Sec. 2) */
} bkm_stats;

/* Fill *p with the defaults listed above for k blocks. */
void bkm_default_params(bkm_params* p, int32_t k);

/* Hilbert space-filling-curve bootstrap (Alg. 2: the curve index of every
 * point, the sort by it and the initial centers; Sec. 4.1).
 *   Key of point i: with lo/hi the global bounding box and ext its largest
 *   extent, cell q_j = min(2^m-1, floor((x_j - lo_j) * (2^m / ext))), then the
 *   order-m Hilbert index of (q_0..q_{d-1}) (Skilling's transpose algorithm,
 *   levels most significant first, axis 0 first within a level).  ext == 0
 *   gives key 0 for every point.
 *   Points are stably sorted by key (ties keep input order) and center c is
 *   the sorted point floor(c*n/k) + floor(n/(2k)).
 * Outputs:
 *   centers_out [device] k*d doubles, row-major [k][d] (FP32 input widened).
 *   perm_out    [device] n int32, sorted position -> input index, or NULL.
 *   keys_out    [device] n uint64, key of each point in input order, or NULL.
 * Errors: BKM_EINVAL, BKM_EDATA (non-finite coordinate), BKM_ENOMEM, BKM_EHIP. */
int bkm_init_centers_sfc(const bkm_points* pts, int32_t k, int32_t hilbert_order,
                         double* centers_out, int32_t* perm_out, uint64_t* keys_out,
                         void* stream);

/* Balanced k-means (Alg. 2 around Alg. 1).
 *   Effective distance dist(p,c)/influence(c), Euclidean, not squared
 *   (Sec. 4.2); each sweep assigns every point the argmin (ties to the lowest
 *   center index), sums block weights, and stops the AssignAndBalance call when
 *   max weight <= L_max, else multiplies influence(c) by
 *   clamp((W/k / weight(c))^(1/d), 0.95, 1.05) (Eq. 1 read so that oversized
 *   blocks lose influence, 5% step limit; an empty block gets 1.05).  After each
 *   call the centers move to the weighted means of their blocks (an empty block
 *   keeps its center); the run stops when the largest move is below
 *   delta_threshold, else the influence is eroded (Sec. 4.2:
 *   alpha = 2/(1+exp(-delta/beta)) - 1, influence <- influence^(1-alpha), beta
 *   the mean bounding-box diagonal of the non-empty blocks) and the next call
 *   starts.  Points are processed in Hilbert order; the Hamerly bounds
 *   (Sec. 4.3) and box pruning (Sec. 4.4) are exact, so the assignment is the
 *   argmin itself.
 * Inputs:
 *   centers_init [device] k*d doubles [k][d], or NULL for the SFC bootstrap.
 * Outputs (device, caller-allocated; NULL skips an optional one):
 *   assignment_out    n int32 block ids in input order (required).
 *   centers_out       k*d doubles [k][d] (required): the final centers.
 *   influence_out     k doubles, or NULL.
 *   block_weights_out k doubles (exact integers for unit weights), or NULL.
 *   info              [host] counters, or NULL.
 * Returns BKM_OK, BKM_WUNBALANCED, or an error code. */
int bkm_balanced_kmeans(const bkm_points* pts, const bkm_params* prm,
                        const double* centers_init, int32_t* assignment_out,
                        double* centers_out, double* influence_out,
                        double* block_weights_out, bkm_info* info, void* stream);

/* Many independent balanced k-means runs (Alg. 2 around Alg. 1, each exactly
 * as bkm_balanced_kmeans with SFC-bootstrap centers) in one call.  Instances
 * may differ in n, k, d, dtype, weights and parameters.  Their bootstraps run
 * side by side on worker streams; then every per-sweep kernel is one launch
 * over all instances that share d, precision, tile size and weighting, each
 * block finding its instance in a block map, and the round loop is captured
 * once in a HIP graph and replayed until every instance is done (a finished
 * instance turns its kernels into no-ops).  Results are identical to
 * count separate bkm_balanced_kmeans calls with the same parameters.
 *   pts   [host] count point sets (device coordinate/weight pointers inside).
 *   prm   [host] count parameter sets; tile_points 0 picks the tile size from
 *         the mean number of points per block; timing is ignored;
 *         sample_init must be 0 (BKM_EINVAL otherwise).
 *   assignment_out [host] count device pointers, n_i int32 each (input order).
 *   centers_out    [host] count device pointers, k_i*d_i doubles each [k][d].
 *   info  [host] count records, or NULL; bootstrap_ms and total_ms are those
 *         of the whole call.
 * Returns BKM_OK when every instance balanced, BKM_WUNBALANCED when some did
 * not (outputs valid), or an error code; bkm_last_error names the instance
 * of an argument or data error.  Workspace for all instances is one
 * stream-ordered allocation on `stream`, released before return. */
int bkm_balanced_kmeans_batched(const bkm_points* pts, const bkm_params* prm, int32_t count,
                                int32_t* const* assignment_out, double* const* centers_out,
                                bkm_info* info, void* stream);

/* A sequence of `steps` assignment sweeps with caller-given centers and
 * influence (the Alg. 1 inner loop with the bound relaxation of Alg. 2
 * between steps).  Step s uses centers[s] and influence[s]; the Hamerly
 * bounds carry over from step to step, relaxed by how far each center moved
 * and how its influence changed, exactly as in bkm_balanced_kmeans.
 *   centers    [device] steps*k*d doubles, [steps][k][d].
 *   influence  [device] steps*k doubles, > 0.
 *   assignment_out [device] steps*n int32, [steps][n], input order.
 *   block_weights_out [device] steps*k doubles, or NULL.
 *   info [host] counters summed over the steps, or NULL.
 * Errors as bkm_balanced_kmeans. */
int bkm_assign_sweeps(const bkm_points* pts, int32_t k, int32_t steps,
                      const double* centers, const double* influence,
                      int32_t precision, int32_t use_bounds, int32_t tile_points,
                      int32_t* assignment_out, double* block_weights_out,
                      bkm_info* info, void* stream);

/* Autotuner of the sweep's tiling.  Tile size (256, 512, 1024) and tiles per
 * super-tile (8, 16, 24, 32) are chosen by timing short balanced k-means runs
 * (3 rounds, twice each, the faster counts) of every combination on a
 * strided sample of at most 2^23 of the points, with k scaled to keep the
 * mean number of points per block; the objective is the device time of the
 * candidate filters and the sweep per sweep.  Choices are cached per (device
 * architecture, d, precision, weighting, octave of n/k, size class of n:
 * below 2^17, 2^20, 2^23, or above): in the process, and, when the environment variable
 * BKM_TUNE_CACHE names a file, in that file (read once, appended to).
 * bkm_balanced_kmeans and bkm_balanced_kmeans_batched use it for
 * tile_points = 0 (the batched call per instance); the random-sample rounds
 * take the n/k rule.  Results never depend on the tiling, only the time.
 *   force  1: measure even if cached (the new choice replaces the old).
 *   out    [host] the choice and, when measured, the timings.
 * Errors as bkm_balanced_kmeans. */
typedef struct {
    int32_t tile_points;      /* chosen tile size */
    int32_t super_tiles;      /* chosen tiles per super-tile (params.super_tiles if set) */
    int32_t from_cache;       /* 1: taken from the cache, nothing measured */
    int32_t candidates;       /* configurations timed */
    double best_us;           /* per-sweep time of the choice on the sample (us) */
    double default_us;        /* per-sweep time of the n/k rule with 16 tiles per super-tile */
    int64_t sample_points;    /* points of the sample */
    int32_t sample_k;         /* blocks of the sample runs */
    int32_t pad;
} bkm_tune_result;

int bkm_autotune(const bkm_points* pts, const bkm_params* prm, int32_t force,
                 bkm_tune_result* out, void* stream);

/* Forgets every cached tuning choice of this process (the cache file is not
 * touched). */
void bkm_autotune_clear(void);

/* Statistics of a given assignment (Sec. 2): block weights, weighted block
 * means (NaN for an empty block), imbalance, k-means objective, empty and
 * overloaded block counts.
 *   assignment [device] n int32 in [0, k).
 *   target_sizes [device] k relative block sizes as in bkm_params, or NULL.
 *   block_weights_out, centers_out [device] k and k*d doubles, or NULL.
 *   out [host] required.
 * Errors: BKM_EINVAL (also for an assignment outside [0,k)), BKM_EDATA,
 * BKM_ENOMEM, BKM_EHIP. */
int bkm_partition_stats(const bkm_points* pts, const int32_t* assignment, int32_t k,
                        double epsilon, const double* target_sizes, double* block_weights_out,
                        double* centers_out, bkm_stats* out, void* stream);

/* bkm_partition_stats without any device or host allocation, for callers
 * that cannot allocate: code under stream capture into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and errors as bkm_partition_stats, plus BKM_EINVAL for k above
 * BKM_NOALLOC_MAX_K.  Its workspace is one static device array of
 * BKM_NOALLOC_SCRATCH_BYTES per device, held from the first call on a device
 * until the process ends; every call on a device shares it, so calls that
 * overlap on one device (different streams or threads) race and must be
 * serialised by the caller.  The call returns after the stream has finished
 * (it fills a host struct). */
#define BKM_NOALLOC_MAX_K 65536
#define BKM_NOALLOC_SCRATCH_BYTES (8 << 20)
int bkm_partition_stats_noalloc(const bkm_points* pts, const int32_t* assignment, int32_t k,
                                double epsilon, const double* target_sizes,
                                double* block_weights_out, double* centers_out, bkm_stats* out,
                                void* stream);

/* ---------------------------------------------------------------------------
 * Graph-quality evaluation (Sec. 2, the block measures; Sec. 5.2, Metrics).
 * The paper measures partitions on the meshes' graphs; these calls build
 * k-nearest-neighbour graphs of point clouds and evaluate any graph given as
 * CSR.
 * ------------------------------------------------------------------------- */

typedef struct {
    int64_t group_visits;     /* point pairs compared / (64 * 64): a query group of 64
                                 points against 64 partners (visits of 8-point parts
                                 count 1/8, rounded down over the call) */
    double layout_ms;         /* device time of the Hilbert tile layout it searches */
    double search_ms;         /* device time of the neighbour search kernel */
} bkm_knn_info;

/* The knn nearest neighbours of every point: the knn points q != p with the
 * smallest (squared Euclidean distance in FP64, ((dx*dx + dy*dy) + dz*dz),
 * input index of q), nearest first.  Exact, not approximate.
 *   knn      1..16, at most n-1.
 *   nbr_out  [device] n*knn int32, [n][knn], input indices.
 *   order_out [device] n int32 or NULL: the input indices in the Hilbert
 *            order the search used, a spatially coherent order to pass to
 *            bkm_knn_graph.
 *   info     [host] or NULL (then no events are recorded).
 * Errors: BKM_EINVAL, BKM_EDATA (non-finite coordinate), BKM_ENOMEM,
 * BKM_EHIP. */
int bkm_knn(const bkm_points* pts, int32_t knn, int32_t* nbr_out, int32_t* order_out,
            bkm_knn_info* info, void* stream);

/* The undirected graph of neighbour lists: edge {p, q} when q is in p's list
 * or p in q's; CSR with both directions, each row sorted ascending.
 *   nbr      [device] n*knn int32 from bkm_knn (or any lists without self
 *            entries).
 *   order    [device] n int32 or NULL: the order in which the passes over
 *            the entries take the vertices, a permutation of 0..n-1
 *            (checked); the result does not depend on it, the speed does: in
 *            a spatially coherent order (bkm_knn's order_out) the vertices
 *            that reread a row come close together in time and hit in cache.
 *   row_ptr_out [device] n+1 int64.
 *   col_out  [device] room for 2*n*knn int32; the first *nnz_out are used.
 *   nnz_out  [host] or NULL.
 * Errors: BKM_EINVAL (also for an entry outside [0, n) or equal to its own
 * row, and an order that is not a permutation), BKM_ENOMEM, BKM_EHIP. */
int bkm_knn_graph(int64_t n, int32_t knn, const int32_t* nbr, const int32_t* order,
                  int64_t* row_ptr_out, int32_t* col_out, int64_t* nnz_out, void* stream);

typedef struct {
    int64_t edge_cut;           /* undirected edges between different blocks */
    int64_t max_comm;           /* max over blocks of comm(V_i) */
    int64_t total_comm;         /* sum over blocks of comm(V_i) */
    int32_t max_diameter;       /* largest finite block diameter bound */
    int32_t disconnected_blocks;
    double harmonic_diameter;   /* harmonic mean of the bounds over blocks of >= 2
                                   vertices (1/inf = 0); inf if all are disconnected,
                                   0 if there are none */
    int32_t bfs_levels;         /* the most breadth-first levels one block's searches ran
                                   (one workgroup per block: every block's first search
                                   in one launch, the connected blocks' others in a
                                   second) */
    int32_t exact_blocks;       /* non-empty connected blocks whose bound is proven exact */
} bkm_graph_stats;

/* Edge cut, communication volume and block diameters of a partition of an
 * undirected graph (Sec. 2 definitions):
 *   comm(V_i) = sum over v in V_i of the number of blocks other than V_i
 *   holding a neighbour of v;
 *   the diameter of a block is bounded from below as in Sec. 5.2 (Metrics),
 *   by the first 3 rounds of the iFUB algorithm (Crescenzi et al., Theor.
 *   Comput. Sci. 514, 2013) inside the block, started from a 4-sweep:
 *   r1 = the block's lowest vertex; a1, b1 = farthest from r1, a1; r2 = the
 *   vertex at distance floor(ecc(a1)/2) from a1 on the a1-b1 path; a2, b2 =
 *   farthest from r2, a2; u = the vertex at distance floor(ecc(a2)/2) from
 *   a2 on the a2-b2 path; l = max(ecc(a1), ecc(a2)).  Farthest = largest
 *   hop distance, lowest index on ties; a path is walked back from its far
 *   end, each step to the lowest-index neighbour one level closer.  iFUB
 *   from u: i = ecc(u), lb = max(l, i), ub = 2i; each round (while ub > lb,
 *   at most 3) takes B = the largest eccentricity of the vertices at
 *   distance i from u; if max(lb, B) > 2(i-1) then lb = ub = max(lb, B),
 *   else lb = max(lb, B), ub = 2(i-1), i = i-1.  The bound is lb (exact
 *   when lb == ub); -1 if the block is disconnected, 0 if it is empty.
 *   row_ptr [device] n+1 int64, col [device] nnz int32: CSR holding both
 *           directions of every edge.
 *   assignment [device] n int32 in [0, k).
 *   comm_out [device] k int64; diameter_out, diameter_ub_out [device] k
 *   int32 (lower bound lb and proven upper bound ub); each may be NULL.
 *   out [host] required.
 * Errors: BKM_EINVAL (also for an assignment, row pointer or column out of
 * range), BKM_ENOMEM, BKM_EHIP. */
int bkm_graph_metrics(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                      const int32_t* assignment, int32_t k, int64_t* comm_out,
                      int32_t* diameter_out, int32_t* diameter_ub_out, bkm_graph_stats* out,
                      void* stream);

/* Message of the last nonzero return on the calling thread ("" if none). */
const char* bkm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BKM_H */
