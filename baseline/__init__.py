"""Pruned FP64 CPU balanced k-means (Hamerly bounds + bounding-box
candidates, OpenMP): the CPU baseline the GPU path is timed against.  Not the
oracle and not part of the library; bench.py and the tests use it.  Built by
baseline/build.py into baseline/libpruned.so."""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpruned.so")
_LIB = None


class PrunedInfo(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("sweeps", C.c_int32), ("balanced", C.c_int32),
                ("converged", C.c_int32), ("evaluated", C.c_int64), ("skipped", C.c_int64),
                ("cand_evals", C.c_int64), ("sweep_seconds", C.c_double),
                ("total_seconds", C.c_double)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with python -m baseline.build")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.pruned_balanced_kmeans.argtypes = [C.c_int64, C.c_int, P, C.c_int, C.c_double, C.c_int,
                                             C.c_int, C.c_double, C.c_int, P, P, P, P,
                                             C.POINTER(PrunedInfo)]
        L.pruned_balanced_kmeans.restype = C.c_int
        L.pruned_num_threads.restype = C.c_int
        L.pruned_set_threads.argtypes = [C.c_int]
        L.pruned_set_threads.restype = None
        _LIB = L
    return _LIB


def num_threads():
    return int(lib().pruned_num_threads())


def set_threads(t):
    lib().pruned_set_threads(int(t))


def balanced_kmeans(X, k, eps, centers_init, max_iter=50, max_balance_iter=20,
                    delta_threshold=None, erosion=True):
    """The oracle's balanced k-means (unit weights) with the paper's exact
    prunings; centers_init [k][d] (the SFC centers).  Returns dict(A,
    centers, influence, info)."""
    X = [np.ascontiguousarray(x, dtype=np.float64) for x in X]
    n, d = len(X[0]), len(X)
    if delta_threshold is None:
        ext = max(float(x.max() - x.min()) for x in X)
        delta_threshold = 1e-5 * ext
    arr = (C.c_void_p * 3)(*[x.ctypes.data for x in X], *([None] * (3 - d)))
    ci = np.ascontiguousarray(centers_init, dtype=np.float64)
    A = np.empty(n, dtype=np.int32)
    cen = np.empty((k, d))
    infl = np.empty(k)
    info = PrunedInfo()
    rc = lib().pruned_balanced_kmeans(n, d, arr, int(k), float(eps), int(max_iter),
                                      int(max_balance_iter), float(delta_threshold),
                                      1 if erosion else 0, ci.ctypes.data, A.ctypes.data,
                                      cen.ctypes.data, infl.ctypes.data, C.byref(info))
    if rc != 0:
        raise RuntimeError(f"pruned_balanced_kmeans failed: {rc}")
    return dict(A=A, centers=cen, influence=infl,
                info={f: getattr(info, f) for f, _ in PrunedInfo._fields_})
