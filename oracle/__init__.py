"""Plain FP64 CPU oracle of balanced k-means (arXiv:1805.01208).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py.  The GPU library never imports it.

Thin ctypes wrapper over ``liboracle.so`` (built from ``bkm_oracle.c`` by
``oracle/build.py``).  Points are passed as a list of d contiguous float64
numpy arrays (SoA); FP32 inputs are widened to FP64 exactly before the call.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None


class OracleInfo(C.Structure):
    _fields_ = [
        ("rounds", C.c_int32), ("sweeps", C.c_int32), ("balanced", C.c_int32),
        ("converged", C.c_int32), ("imbalance", C.c_double),
        ("max_block_weight", C.c_double), ("lmax", C.c_double),
    ]


class OracleStats(C.Structure):
    _fields_ = [
        ("imbalance", C.c_double), ("objective", C.c_double), ("lmax", C.c_double),
        ("empty_blocks", C.c_int32), ("overloaded_blocks", C.c_int32),
    ]


class OracleGraphStats(C.Structure):
    _fields_ = [
        ("edge_cut", C.c_int64), ("max_comm", C.c_int64), ("total_comm", C.c_int64),
        ("max_diameter", C.c_int32), ("disconnected_blocks", C.c_int32),
        ("exact_blocks", C.c_int32), ("harmonic_diameter", C.c_double),
    ]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P, D, I64, I32 = C.c_void_p, C.c_double, C.c_int64, C.c_int32
        L.oracle_bbox.argtypes = [I64, C.c_int, P, P, P]
        L.oracle_hilbert_index.argtypes = [P, C.c_int, C.c_int]
        L.oracle_hilbert_index.restype = C.c_uint64
        L.oracle_sfc_keys.argtypes = [I64, C.c_int, P, C.c_int, P]
        L.oracle_sfc_order.argtypes = [I64, P, P]
        L.oracle_init_centers_sfc.argtypes = [I64, C.c_int, P, C.c_int, C.c_int, P, P, P, P]
        L.oracle_assign.argtypes = [I64, C.c_int, P, C.c_int, P, P, P, P, P]
        L.oracle_block_weights.argtypes = [I64, P, P, C.c_int, P]
        L.oracle_total_weight.argtypes = [I64, P]
        L.oracle_total_weight.restype = D
        L.oracle_lmax.argtypes = [I64, C.c_int, D, D, C.c_int]
        L.oracle_lmax.restype = D
        L.oracle_balance_step.argtypes = [C.c_int, C.c_int, P, D, D, P]
        L.oracle_balance_step_targets.argtypes = [C.c_int, C.c_int, P, P, P, P]
        L.oracle_targets.argtypes = [I64, C.c_int, D, D, C.c_int, P, P, P]
        L.oracle_new_centers.argtypes = [I64, C.c_int, P, P, P, C.c_int, P, P, P]
        L.oracle_beta.argtypes = [I64, C.c_int, P, P, C.c_int]
        L.oracle_beta.restype = D
        L.oracle_erode.argtypes = [C.c_int, P, D, P]
        L.oracle_erode.restype = None
        L.oracle_balanced_kmeans.argtypes = [
            I64, C.c_int, P, P, C.c_int, D, C.c_int, C.c_int, D, C.c_int, C.c_int,
            P, P, P, P, P, P, P, P, C.POINTER(OracleInfo)]
        L.oracle_balanced_kmeans_sampled.argtypes = [
            I64, C.c_int, P, P, C.c_int, D, C.c_int, C.c_int, D, C.c_int, C.c_int,
            I64, P, P, P, P, P, P, P, C.POINTER(OracleInfo), P, P]
        L.oracle_partition_stats.argtypes = [
            I64, C.c_int, P, P, P, C.c_int, D, P, P, P, C.POINTER(OracleStats)]
        L.oracle_knn.argtypes = [I64, C.c_int, P, C.c_int, P]
        L.oracle_knn_of.argtypes = [I64, C.c_int, P, C.c_int, I64, P, P]
        L.oracle_knn_symmetrize.argtypes = [I64, C.c_int, P, P, P, P]
        L.oracle_graph_metrics.argtypes = [I64, P, P, P, C.c_int, P, P, P,
                                           C.POINTER(OracleGraphStats)]
        L.oracle_ifub_trace.argtypes = [I64, P, P, P]
        L.oracle_num_threads.argtypes = []
        _ = I32
        _LIB = L
    return _LIB


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Points:
    """Keeps the contiguous FP64 SoA arrays alive and exposes a double** ."""

    def __init__(self, X):
        self.cols = [np.ascontiguousarray(np.asarray(c, dtype=np.float64)) for c in X]
        self.n = int(self.cols[0].shape[0])
        self.d = len(self.cols)
        self.arr = (C.c_void_p * 3)(*[c.ctypes.data for c in self.cols] + [None] * (3 - self.d))


def _weights(W):
    return None if W is None else np.ascontiguousarray(np.asarray(W, dtype=np.float64))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def bbox(X):
    p = _Points(X)
    lo = np.zeros(3)
    hi = np.zeros(3)
    _check(lib().oracle_bbox(p.n, p.d, p.arr, _ptr(lo), _ptr(hi)), "bbox")
    return lo[:p.d], hi[:p.d]


def hilbert_index(q, m):
    q = np.ascontiguousarray(np.asarray(q, dtype=np.uint32))
    return int(lib().oracle_hilbert_index(_ptr(q), int(q.shape[0]), int(m)))


def hilbert_indices(Q, m):
    """Keys of integer cells Q ([N][d]) at order m."""
    Q = np.asarray(Q, dtype=np.uint32)
    return np.array([hilbert_index(q, m) for q in Q], dtype=np.uint64)


def sfc_keys(X, m):
    p = _Points(X)
    keys = np.empty(p.n, dtype=np.uint64)
    _check(lib().oracle_sfc_keys(p.n, p.d, p.arr, int(m), _ptr(keys)), "sfc_keys")
    return keys


def sfc_order(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    perm = np.empty(keys.shape[0], dtype=np.int64)
    _check(lib().oracle_sfc_order(keys.shape[0], _ptr(keys), _ptr(perm)), "sfc_order")
    return perm


def _targets(t, k):
    if t is None:
        return None
    t = np.ascontiguousarray(t, dtype=np.float64)
    if t.shape != (k,):
        raise ValueError("target_sizes must hold k values")
    return t


def init_centers_sfc(X, k, m, target_sizes=None):
    """Returns (centers [k][d], perm sorted->original, keys original order)."""
    p = _Points(X)
    centers = np.empty((k, p.d), dtype=np.float64)
    perm = np.empty(p.n, dtype=np.int64)
    keys = np.empty(p.n, dtype=np.uint64)
    t = _targets(target_sizes, k)
    _check(lib().oracle_init_centers_sfc(p.n, p.d, p.arr, int(k), int(m), _ptr(t),
                                         _ptr(centers), _ptr(perm), _ptr(keys)),
           "init_centers_sfc")
    return centers, perm, keys


def assign(X, centers, influence):
    """Brute-force argmin of the effective distance: (A, best, second)."""
    p = _Points(X)
    centers = np.ascontiguousarray(centers, dtype=np.float64)
    influence = np.ascontiguousarray(influence, dtype=np.float64)
    k = centers.shape[0]
    A = np.empty(p.n, dtype=np.int32)
    best = np.empty(p.n)
    second = np.empty(p.n)
    _check(lib().oracle_assign(p.n, p.d, p.arr, k, _ptr(centers), _ptr(influence), _ptr(A),
                               _ptr(best), _ptr(second)), "assign")
    return A, best, second


def block_weights(A, W, k):
    A = np.ascontiguousarray(A, dtype=np.int32)
    W = _weights(W)
    out = np.empty(k)
    _check(lib().oracle_block_weights(A.shape[0], _ptr(A), _ptr(W), int(k), _ptr(out)),
           "block_weights")
    return out


def total_weight(n, W):
    W = _weights(W)
    return float(lib().oracle_total_weight(int(n), _ptr(W)))


def lmax(n, k, eps, W=None):
    return float(lib().oracle_lmax(int(n), int(k), float(eps), total_weight(n, W), W is None))


def targets(n, k, eps, W=None, target_sizes=None):
    """Per-block targets T_c and limits L_max,c: (T, L)."""
    T = np.empty(k)
    L = np.empty(k)
    t = _targets(target_sizes, k)
    _check(lib().oracle_targets(int(n), int(k), float(eps), total_weight(n, W), W is None,
                                _ptr(t), _ptr(T), _ptr(L)), "targets")
    return T, L


def balance_step_targets(sizes, d, L, T, influence):
    """Balance test + influence update with a limit and target per block."""
    sizes = np.ascontiguousarray(sizes, dtype=np.float64)
    L = np.ascontiguousarray(L, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    infl = np.array(influence, dtype=np.float64, copy=True)
    b = lib().oracle_balance_step_targets(sizes.shape[0], int(d), _ptr(sizes), _ptr(L), _ptr(T),
                                          _ptr(infl))
    return bool(b), infl


def balance_step(sizes, d, lmax_value, target, influence):
    """One balance test + influence update; returns (balanced, new influence)."""
    sizes = np.ascontiguousarray(sizes, dtype=np.float64)
    infl = np.array(influence, dtype=np.float64, copy=True)
    b = lib().oracle_balance_step(sizes.shape[0], int(d), _ptr(sizes), float(lmax_value),
                                  float(target), _ptr(infl))
    return bool(b), infl


def new_centers(X, W, A, centers_old):
    p = _Points(X)
    W = _weights(W)
    A = np.ascontiguousarray(A, dtype=np.int32)
    centers_old = np.ascontiguousarray(centers_old, dtype=np.float64)
    k = centers_old.shape[0]
    cn = np.empty_like(centers_old)
    delta = np.empty(k)
    _check(lib().oracle_new_centers(p.n, p.d, p.arr, _ptr(W), _ptr(A), k, _ptr(centers_old),
                                    _ptr(cn), _ptr(delta)), "new_centers")
    return cn, delta


def beta(X, A, k):
    p = _Points(X)
    A = np.ascontiguousarray(A, dtype=np.int32)
    return float(lib().oracle_beta(p.n, p.d, p.arr, _ptr(A), int(k)))


def erode(delta, beta_value, influence):
    delta = np.ascontiguousarray(delta, dtype=np.float64)
    infl = np.array(influence, dtype=np.float64, copy=True)
    lib().oracle_erode(delta.shape[0], _ptr(delta), float(beta_value), _ptr(infl))
    return infl


def balanced_kmeans(X, k, eps, W=None, max_iter=50, max_balance_iter=20,
                    delta_threshold=None, hilbert_order=16, centers_init=None,
                    influence_init=None, sample_keys=None, sample_start=0,
                    target_sizes=None, erosion=True):
    """Full balanced k-means.  delta_threshold None -> 1e-5 * largest bbox extent.
    With sample_keys (one uint64 per point) the run starts with the
    random-sample initialization over the order of (key, index), from
    sample_start points (0: 100 per block, 100 * k).
    target_sizes: k relative block sizes, or None for equal blocks.

    Returns dict(A, centers, influence, block_weights, sweeps_per_round, info)."""
    p = _Points(X)
    W = _weights(W)
    if delta_threshold is None:
        lo, hi = bbox(X)
        delta_threshold = 1e-5 * float(np.max(hi - lo))
    A = np.empty(p.n, dtype=np.int32)
    centers = np.empty((k, p.d))
    infl = np.empty(k)
    bw = np.empty(k)
    spr = np.zeros(max_iter, dtype=np.int32)
    info = OracleInfo()
    extra = {}
    t = _targets(target_sizes, k)
    if sample_keys is None:
        ci = None if centers_init is None else np.ascontiguousarray(centers_init, dtype=np.float64)
        ii = None if influence_init is None else np.ascontiguousarray(influence_init, dtype=np.float64)
        _check(lib().oracle_balanced_kmeans(
            p.n, p.d, p.arr, _ptr(W), int(k), float(eps), int(max_iter), int(max_balance_iter),
            float(delta_threshold), int(hilbert_order), 1 if erosion else 0, _ptr(ci), _ptr(ii),
            _ptr(t), _ptr(A),
            _ptr(centers), _ptr(infl), _ptr(bw), _ptr(spr), C.byref(info)), "balanced_kmeans")
    else:
        keys = np.ascontiguousarray(sample_keys, dtype=np.uint64)
        sr = np.zeros(1, dtype=np.int32)
        ss = np.zeros(1, dtype=np.int32)
        _check(lib().oracle_balanced_kmeans_sampled(
            p.n, p.d, p.arr, _ptr(W), int(k), float(eps), int(max_iter), int(max_balance_iter),
            float(delta_threshold), int(hilbert_order), 1 if erosion else 0, int(sample_start),
            _ptr(keys), _ptr(t),
            _ptr(A),
            _ptr(centers), _ptr(infl), _ptr(bw), _ptr(spr), C.byref(info), _ptr(sr), _ptr(ss)),
            "balanced_kmeans_sampled")
        extra = dict(sample_rounds=int(sr[0]), sample_sweeps=int(ss[0]))
    out = dict(A=A, centers=centers, influence=infl, block_weights=bw,
               sweeps_per_round=spr[:info.rounds].copy(),
               info={f: getattr(info, f) for f, _ in OracleInfo._fields_})
    out["info"].update(extra)
    return out


def partition_stats(X, A, k, eps, W=None, target_sizes=None):
    p = _Points(X)
    t = _targets(target_sizes, k)
    W = _weights(W)
    A = np.ascontiguousarray(A, dtype=np.int32)
    bw = np.empty(k)
    centers = np.empty((k, p.d))
    st = OracleStats()
    _check(lib().oracle_partition_stats(p.n, p.d, p.arr, _ptr(W), _ptr(A), int(k), float(eps),
                                        _ptr(t), _ptr(bw), _ptr(centers), C.byref(st)), "partition_stats")
    return dict(block_weights=bw, centers=centers,
                **{f: getattr(st, f) for f, _ in OracleStats._fields_})


# ---------------------------------------------------------------- graph quality
def knn(X, K):
    """K nearest neighbours of every point, [n][K] input indices, nearest first."""
    p = _Points(X)
    nbr = np.empty((p.n, int(K)), dtype=np.int32)
    _check(lib().oracle_knn(p.n, p.d, p.arr, int(K), _ptr(nbr)), "knn")
    return nbr


def knn_of(X, K, queries):
    """K nearest neighbours (over all points) of the given query points."""
    p = _Points(X)
    q = np.ascontiguousarray(queries, dtype=np.int64)
    nbr = np.empty((q.shape[0], int(K)), dtype=np.int32)
    _check(lib().oracle_knn_of(p.n, p.d, p.arr, int(K), q.shape[0], _ptr(q), _ptr(nbr)), "knn_of")
    return nbr


def knn_symmetrize(nbr):
    """Undirected graph of neighbour lists as CSR: (row_ptr int64[n+1], col int32[nnz])."""
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    n, K = nbr.shape
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(2 * n * K, dtype=np.int32)
    nnz = np.zeros(1, dtype=np.int64)
    _check(lib().oracle_knn_symmetrize(n, K, _ptr(nbr), _ptr(row_ptr), _ptr(col), _ptr(nnz)),
           "knn_symmetrize")
    return row_ptr, col[:int(nnz[0])].copy()


def graph_metrics(row_ptr, col, A, k):
    """Edge cut, communication volumes and block diameter bounds of A."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    A = np.ascontiguousarray(A, dtype=np.int32)
    n = A.shape[0]
    comm = np.empty(k, dtype=np.int64)
    diam = np.empty(k, dtype=np.int32)
    dub = np.empty(k, dtype=np.int32)
    st = OracleGraphStats()
    _check(lib().oracle_graph_metrics(n, _ptr(row_ptr), _ptr(col), _ptr(A), int(k), _ptr(comm),
                                      _ptr(diam), _ptr(dub), C.byref(st)), "graph_metrics")
    out = {f: getattr(st, f) for f, _ in OracleGraphStats._fields_}
    out.update(comm=comm, diameter=diam, diameter_ub=dub)
    return out


def ifub_trace(row_ptr, col):
    """The steps of the diameter bound (4-sweep, then up to 3 iFUB rounds) on
    a connected graph taken as one block: dict of a1, b1, r2, a2, b2, u, l,
    rounds, lb, ub."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    t = np.zeros(10, dtype=np.int64)
    _check(lib().oracle_ifub_trace(row_ptr.shape[0] - 1, _ptr(row_ptr), _ptr(col), _ptr(t)),
           "ifub_trace")
    return dict(zip(("a1", "b1", "r2", "a2", "b2", "u", "l", "rounds", "lb", "ub"),
                    (int(v) for v in t)))
