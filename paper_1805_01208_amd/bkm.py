"""Thin ctypes binding of libbkm (include/bkm.h).

Argument marshalling only: every step runs in the HIP kernels of libbkm.so.
Points are a list of d contiguous CUDA tensors (float32 or float64, same dtype,
input order); weights a float64 CUDA tensor or None.  Work is enqueued on
torch's current stream.  There is no CPU fallback: a missing library raises.
"""
import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbkm.so")

BKM_OK, BKM_EINVAL, BKM_EDATA, BKM_ENOMEM, BKM_EHIP, BKM_EINTERNAL = 0, -1, -2, -3, -4, -5
BKM_WUNBALANCED = 1
BKM_F32, BKM_F64 = 0, 1
PREC_F64, PREC_F32_RECHECK = 0, 1
PRECISIONS = {"f64": PREC_F64, "f32_recheck": PREC_F32_RECHECK}


class Points(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("dtype", C.c_int32),
                ("coords", C.c_void_p * 3), ("weights", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("max_iter", C.c_int32), ("max_balance_iter", C.c_int32),
                ("hilbert_order", C.c_int32), ("precision", C.c_int32),
                ("use_bounds", C.c_int32), ("tile_points", C.c_int32),
                ("super_tiles", C.c_int32), ("timing", C.c_int32), ("sample_init", C.c_int32),
                ("erosion", C.c_int32),
                ("epsilon", C.c_double), ("delta_threshold", C.c_double),
                ("recheck_rel_gap", C.c_double), ("sample_start", C.c_int64),
                ("seed", C.c_uint64), ("sample_keys", C.c_void_p),
                ("target_sizes", C.c_void_p), ("debug_checks", C.c_int32), ("pad_", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("sweeps", C.c_int32), ("balanced", C.c_int32),
                ("converged", C.c_int32), ("imbalance", C.c_double),
                ("max_block_weight", C.c_double), ("l_max", C.c_double),
                ("evaluated", C.c_int64), ("skipped", C.c_int64), ("rechecked", C.c_int64),
                ("changed", C.c_int64), ("candidate_evals", C.c_int64),
                ("overflow_tiles", C.c_int64),
                ("bootstrap_ms", C.c_double), ("total_ms", C.c_double),
                ("cand_ms", C.c_double), ("sweep_ms", C.c_double), ("balance_ms", C.c_double),
                ("boxes_ms", C.c_double), ("move_ms", C.c_double),
                ("sample_rounds", C.c_int32), ("sample_sweeps", C.c_int32),
                ("debug_checked", C.c_int64), ("debug_violations", C.c_int64),
                ("list_builds", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("imbalance", C.c_double), ("objective", C.c_double), ("l_max", C.c_double),
                ("empty_blocks", C.c_int32), ("overloaded_blocks", C.c_int32)]


class GraphStats(C.Structure):
    _fields_ = [("edge_cut", C.c_int64), ("max_comm", C.c_int64), ("total_comm", C.c_int64),
                ("max_diameter", C.c_int32), ("disconnected_blocks", C.c_int32),
                ("harmonic_diameter", C.c_double), ("bfs_levels", C.c_int32),
                ("exact_blocks", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("tile_points", C.c_int32), ("super_tiles", C.c_int32),
                ("from_cache", C.c_int32), ("candidates", C.c_int32), ("best_us", C.c_double),
                ("default_us", C.c_double), ("sample_points", C.c_int64),
                ("sample_k", C.c_int32), ("pad", C.c_int32)]


class KnnInfo(C.Structure):
    _fields_ = [("group_visits", C.c_int64), ("layout_ms", C.c_double), ("search_ms", C.c_double)]


class BkmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbkm error {code}: {msg}")
        self.code = code


_LIB = None
FUNCTIONS = ("bkm_default_params", "bkm_init_centers_sfc", "bkm_balanced_kmeans",
             "bkm_balanced_kmeans_batched", "bkm_assign_sweeps", "bkm_partition_stats",
             "bkm_partition_stats_noalloc", "bkm_knn", "bkm_knn_graph", "bkm_graph_metrics",
             "bkm_autotune", "bkm_autotune_clear", "bkm_last_error")


def lib():
    """Load libbkm.so (built by paper_1805_01208_amd/build.py)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "python -m paper_1805_01208_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.bkm_default_params.argtypes = [C.POINTER(Params), C.c_int32]
        L.bkm_default_params.restype = None
        L.bkm_init_centers_sfc.argtypes = [C.POINTER(Points), C.c_int32, C.c_int32, P, P, P, P]
        L.bkm_balanced_kmeans.argtypes = [C.POINTER(Points), C.POINTER(Params), P, P, P, P, P,
                                          C.POINTER(Info), P]
        L.bkm_assign_sweeps.argtypes = [C.POINTER(Points), C.c_int32, C.c_int32, P, P, C.c_int32,
                                        C.c_int32, C.c_int32, P, P, C.POINTER(Info), P]
        L.bkm_partition_stats.argtypes = [C.POINTER(Points), P, C.c_int32, C.c_double, P, P, P,
                                          C.POINTER(Stats), P]
        L.bkm_partition_stats_noalloc.argtypes = L.bkm_partition_stats.argtypes
        L.bkm_balanced_kmeans_batched.argtypes = [C.POINTER(Points), C.POINTER(Params), C.c_int32,
                                                  C.POINTER(P), C.POINTER(P), C.POINTER(Info), P]
        L.bkm_knn.argtypes = [C.POINTER(Points), C.c_int32, P, P, C.POINTER(KnnInfo), P]
        L.bkm_knn_graph.argtypes = [C.c_int64, C.c_int32, P, P, P, P, C.POINTER(C.c_int64), P]
        L.bkm_graph_metrics.argtypes = [C.c_int64, C.c_int64, P, P, P, C.c_int32, P, P, P,
                                        C.POINTER(GraphStats), P]
        L.bkm_autotune.argtypes = [C.POINTER(Points), C.POINTER(Params), C.c_int32,
                                   C.POINTER(TuneResult), P]
        L.bkm_autotune_clear.argtypes = []
        L.bkm_autotune_clear.restype = None
        L.bkm_last_error.argtypes = []
        L.bkm_last_error.restype = C.c_char_p
        for f in ("bkm_init_centers_sfc", "bkm_balanced_kmeans", "bkm_assign_sweeps",
                  "bkm_partition_stats", "bkm_partition_stats_noalloc",
                  "bkm_balanced_kmeans_batched", "bkm_knn",
                  "bkm_knn_graph", "bkm_graph_metrics", "bkm_autotune"):
            getattr(L, f).restype = C.c_int
        _LIB = L
    return _LIB


def _check(rc):
    if rc < 0:
        raise BkmError(rc, lib().bkm_last_error().decode())
    return rc


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_points(X, W=None):
    """Points struct over caller tensors (kept alive by the caller)."""
    X = list(X)
    d = len(X)
    if d not in (2, 3):
        raise ValueError("points need 2 or 3 coordinate arrays")
    dt = X[0].dtype
    for x in X:
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous() or x.dim() != 1:
            raise ValueError("coordinates must be contiguous 1-D CUDA tensors of one dtype")
    if dt not in (torch.float32, torch.float64):
        raise ValueError("coordinates must be float32 or float64")
    if W is not None and (W.dtype != torch.float64 or not W.is_cuda or not W.is_contiguous()):
        raise ValueError("weights must be a contiguous float64 CUDA tensor")
    p = Points()
    p.n = X[0].numel()
    p.d = d
    p.dtype = BKM_F32 if dt == torch.float32 else BKM_F64
    for j in range(3):
        p.coords[j] = X[j].data_ptr() if j < d else None
    p.weights = None if W is None else W.data_ptr()
    return p


def default_params(k):
    p = Params()
    lib().bkm_default_params(C.byref(p), int(k))
    return p


def info_dict(info):
    return {f: getattr(info, f) for f, _ in Info._fields_}


def init_centers_sfc(X, k, hilbert_order=16):
    """(centers [k,d] float64, perm int32 sorted->input, keys int64 bit pattern of uint64)."""
    dev = X[0].device
    pts = make_points(X)
    cen = torch.empty((k, pts.d), dtype=torch.float64, device=dev)
    perm = torch.empty(pts.n, dtype=torch.int32, device=dev)
    keys = torch.empty(pts.n, dtype=torch.int64, device=dev)
    _check(lib().bkm_init_centers_sfc(C.byref(pts), int(k), int(hilbert_order), _ptr(cen),
                                      _ptr(perm), _ptr(keys), _stream()))
    return cen, perm, keys


def _targets(t, k, dev):
    """Target sizes as a contiguous float64 device tensor of k values, or None."""
    if t is None:
        return None
    t = torch.as_tensor(t, dtype=torch.float64).to(device=dev).contiguous()
    if t.numel() != k:
        raise ValueError("target_sizes must hold k values")
    return t


def balanced_kmeans(X, k, W=None, eps=0.03, max_iter=50, max_balance_iter=20,
                    delta_threshold=-1.0, hilbert_order=16, precision="f32_recheck",
                    use_bounds=True, tile_points=0, super_tiles=0, recheck_rel_gap=1e-5,
                    centers_init=None, timing=False, out=None, sample_init=False,
                    sample_start=0, seed=0, sample_keys=None, target_sizes=None,
                    erosion=True, debug_checks=0):
    """Balanced k-means; returns dict(A, centers, influence, block_weights, info, code).
    sample_init: start with rounds on random samples doubling from sample_start
    points (0: 100 per block, i.e. 100 * k), ordered by splitmix64(seed, index)
    or by sample_keys (n uint64 keys on the device).  target_sizes: k relative
    block sizes (device tensor), or None for equal blocks."""
    dev = X[0].device
    pts = make_points(X, W)
    prm = default_params(k)
    prm.epsilon = float(eps)
    prm.max_iter = int(max_iter)
    prm.max_balance_iter = int(max_balance_iter)
    prm.delta_threshold = float(delta_threshold)
    prm.hilbert_order = int(hilbert_order)
    prm.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prm.use_bounds = 1 if use_bounds else 0
    prm.tile_points = int(tile_points)
    prm.super_tiles = int(super_tiles)
    prm.recheck_rel_gap = float(recheck_rel_gap)
    prm.timing = 1 if timing else 0
    prm.sample_init = 1 if sample_init else 0
    prm.erosion = 1 if erosion else 0
    prm.debug_checks = int(debug_checks)
    prm.sample_start = int(sample_start)
    prm.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    sk = None
    if sample_keys is not None:
        if sample_keys.numel() != pts.n or sample_keys.element_size() != 8:
            raise ValueError("sample_keys must hold n 64-bit keys")
        sk = sample_keys.to(device=dev).contiguous()
        prm.sample_keys = sk.data_ptr()
    ts = _targets(target_sizes, k, dev)
    prm.target_sizes = None if ts is None else ts.data_ptr()
    if out is None:
        out = dict(A=torch.empty(pts.n, dtype=torch.int32, device=dev),
                   centers=torch.empty((k, pts.d), dtype=torch.float64, device=dev),
                   influence=torch.empty(k, dtype=torch.float64, device=dev),
                   block_weights=torch.empty(k, dtype=torch.float64, device=dev))
    ci = None
    if centers_init is not None:
        ci = centers_init.to(device=dev, dtype=torch.float64).contiguous()
    info = Info()
    rc = _check(lib().bkm_balanced_kmeans(C.byref(pts), C.byref(prm), _ptr(ci), _ptr(out["A"]),
                                          _ptr(out["centers"]), _ptr(out["influence"]),
                                          _ptr(out["block_weights"]), C.byref(info), _stream()))
    res = dict(out)
    res["info"] = info_dict(info)
    res["code"] = rc
    return res


def balanced_kmeans_batched(instances, eps=0.03, max_iter=50, max_balance_iter=20,
                            delta_threshold=-1.0, hilbert_order=16, precision="f32_recheck",
                            use_bounds=True, tile_points=0, super_tiles=0, recheck_rel_gap=1e-5,
                            target_sizes=None, erosion=True):
    """Many balanced k-means runs in one call.  instances: list of (X, k) or
    (X, k, W) with X a list of d device tensors.  Scalar parameters apply to
    every instance; a list gives one value per instance (target_sizes: a
    list of per-instance tensors or None).  Returns a list of dict(A,
    centers, info) and the call's return code."""
    m = len(instances)

    def per(v, i):
        return v[i] if isinstance(v, (list, tuple)) else v

    pts = (Points * m)()
    prm = (Params * m)()
    outs = []
    keep = []
    for i, inst in enumerate(instances):
        X, k = inst[0], int(inst[1])
        W = inst[2] if len(inst) > 2 else None
        pts[i] = make_points(X, W)
        p = default_params(k)
        p.epsilon = float(per(eps, i))
        p.max_iter = int(per(max_iter, i))
        p.max_balance_iter = int(per(max_balance_iter, i))
        p.delta_threshold = float(per(delta_threshold, i))
        p.hilbert_order = int(per(hilbert_order, i))
        pr = per(precision, i)
        p.precision = PRECISIONS[pr] if isinstance(pr, str) else int(pr)
        p.use_bounds = 1 if per(use_bounds, i) else 0
        p.tile_points = int(per(tile_points, i))
        p.super_tiles = int(per(super_tiles, i))
        p.recheck_rel_gap = float(per(recheck_rel_gap, i))
        p.erosion = 1 if per(erosion, i) else 0
        dev = X[0].device
        ts = _targets(None if target_sizes is None else target_sizes[i], k, dev)
        keep.append(ts)
        p.target_sizes = None if ts is None else ts.data_ptr()
        prm[i] = p
        outs.append(dict(A=torch.empty(pts[i].n, dtype=torch.int32, device=dev),
                         centers=torch.empty((k, pts[i].d), dtype=torch.float64, device=dev)))
    asg = (C.c_void_p * m)(*[o["A"].data_ptr() for o in outs])
    cen = (C.c_void_p * m)(*[o["centers"].data_ptr() for o in outs])
    info = (Info * m)()
    rc = _check(lib().bkm_balanced_kmeans_batched(pts, prm, m, asg, cen, info, _stream()))
    for i, o in enumerate(outs):
        o["info"] = info_dict(info[i])
    return outs, rc


def assign_sweeps(X, centers_seq, influence_seq, precision="f32_recheck", use_bounds=True,
                  tile_points=0):
    """Successive sweeps with given (centers [S,k,d], influence [S,k]); returns
    (A [S,n] int32, block weights [S,k] float64, info)."""
    dev = X[0].device
    pts = make_points(X)
    cs = centers_seq.to(device=dev, dtype=torch.float64).contiguous()
    ins = influence_seq.to(device=dev, dtype=torch.float64).contiguous()
    S, k = ins.shape
    A = torch.empty((S, pts.n), dtype=torch.int32, device=dev)
    bw = torch.empty((S, k), dtype=torch.float64, device=dev)
    info = Info()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().bkm_assign_sweeps(C.byref(pts), int(k), int(S), _ptr(cs), _ptr(ins), prec,
                                   1 if use_bounds else 0, int(tile_points), _ptr(A), _ptr(bw),
                                   C.byref(info), _stream()))
    return A, bw, info_dict(info)


def autotune(X, k, W=None, precision="f32_recheck", force=False, super_tiles=0, **kw):
    """The autotuner's tiling for these points (cached, or measured now):
    dict of the bkm_tune_result fields."""
    pts = make_points(X, W)
    prm = default_params(k)
    prm.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    prm.super_tiles = int(super_tiles)
    for f, v in kw.items():
        setattr(prm, f, v)
    res = TuneResult()
    _check(lib().bkm_autotune(C.byref(pts), C.byref(prm), 1 if force else 0, C.byref(res),
                              _stream()))
    return {f: getattr(res, f) for f, _ in TuneResult._fields_ if f != "pad"}


def autotune_clear():
    lib().bkm_autotune_clear()


def partition_stats(X, A, k, eps=0.03, W=None, target_sizes=None):
    dev = X[0].device
    pts = make_points(X, W)
    ts = _targets(target_sizes, k, dev)
    bw = torch.empty(k, dtype=torch.float64, device=dev)
    cen = torch.empty((k, pts.d), dtype=torch.float64, device=dev)
    st = Stats()
    _check(lib().bkm_partition_stats(C.byref(pts), _ptr(A.contiguous()), int(k), float(eps),
                                     _ptr(ts), _ptr(bw), _ptr(cen), C.byref(st), _stream()))
    res = {f: getattr(st, f) for f, _ in Stats._fields_}
    res.update(block_weights=bw, centers=cen)
    return res


def partition_stats_noalloc(X, A, k, eps=0.03, W=None, target_sizes=None, bw=None, cen=None):
    """partition_stats through the no-allocation entry point; bw [k] and cen
    [k, d] float64 device tensors may be passed in (allocated here if not)."""
    dev = X[0].device
    pts = make_points(X, W)
    ts = _targets(target_sizes, k, dev)
    if bw is None:
        bw = torch.empty(k, dtype=torch.float64, device=dev)
    if cen is None:
        cen = torch.empty((k, pts.d), dtype=torch.float64, device=dev)
    st = Stats()
    _check(lib().bkm_partition_stats_noalloc(C.byref(pts), _ptr(A.contiguous()), int(k),
                                             float(eps), _ptr(ts), _ptr(bw), _ptr(cen),
                                             C.byref(st), _stream()))
    res = {f: getattr(st, f) for f, _ in Stats._fields_}
    res.update(block_weights=bw, centers=cen)
    return res


def knn(X, K, order=False):
    """Exact K nearest neighbours of every point: (nbr [n][K] int32 device
    tensor, input indices nearest first; dict(group_visits, layout_ms,
    search_ms)).  With order=True the dict also holds "order", the input
    indices in the search's Hilbert order (for knn_graph)."""
    dev = X[0].device
    pts = make_points(X)
    nbr = torch.empty((pts.n, int(K)), dtype=torch.int32, device=dev)
    o = torch.empty(pts.n, dtype=torch.int32, device=dev) if order else None
    info = KnnInfo()
    _check(lib().bkm_knn(C.byref(pts), int(K), _ptr(nbr), _ptr(o), C.byref(info), _stream()))
    res = {f: getattr(info, f) for f, _ in KnnInfo._fields_}
    if order:
        res["order"] = o
    return nbr, res


def knn_graph(nbr, order=None):
    """Undirected graph of neighbour lists as CSR: (row_ptr int64, col int32).
    `order` (a permutation of 0..n-1, e.g. knn's order) only sets the order
    in which the vertices are processed."""
    n, K = nbr.shape
    dev = nbr.device
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(2 * n * K, dtype=torch.int32, device=dev)
    nnz = C.c_int64(0)
    o = None if order is None else order.to(torch.int32).contiguous()
    _check(lib().bkm_knn_graph(n, K, _ptr(nbr.contiguous()), _ptr(o), _ptr(row_ptr), _ptr(col),
                               C.byref(nnz), _stream()))
    return row_ptr, col[:nnz.value]


def graph_metrics(row_ptr, col, A, k):
    """Edge cut, communication volumes and block diameter bounds of A."""
    dev = A.device
    n = A.numel()
    comm = torch.empty(k, dtype=torch.int64, device=dev)
    diam = torch.empty(k, dtype=torch.int32, device=dev)
    dub = torch.empty(k, dtype=torch.int32, device=dev)
    st = GraphStats()
    _check(lib().bkm_graph_metrics(n, col.numel(), _ptr(row_ptr.contiguous()),
                                   _ptr(col.contiguous()), _ptr(A.contiguous()), int(k),
                                   _ptr(comm), _ptr(diam), _ptr(dub), C.byref(st), _stream()))
    res = {f: getattr(st, f) for f, _ in GraphStats._fields_}
    res.update(comm=comm, diameter=diam, diameter_ub=dub)
    return res
