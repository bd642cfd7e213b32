"""Helpers of the GPU parity tests (not a test module)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

TIE_GAP = 1e-12        # assignments may differ only where the oracle's relative gap is below this
CENTER_RTOL = 1e-10    # centers: relative to max(|C|_inf, bounding-box extent)


def cuda(X, dtype=None):
    out = []
    for x in X:
        t = torch.from_numpy(np.ascontiguousarray(x))
        if dtype is not None:
            t = t.to(dtype)
        out.append(t.cuda())
    return out


def widened(X):
    return [np.asarray(x, dtype=np.float64) for x in X]


def effective_distance(X, C, I, A):
    """eff(p, A[p]) = sqrt(((dx*dx + dy*dy) + dz*dz)) / I[A[p]] in FP64, in the
    oracle's order of operations (numpy does not contract)."""
    A = np.asarray(A, dtype=np.int64)
    s = np.zeros(len(X[0]))
    for j, x in enumerate(X):
        dx = np.asarray(x, dtype=np.float64) - C[A, j]
        s = s + dx * dx
    return np.sqrt(s) / I[A]


def assert_assignment_parity(A_gpu, A_orc, best, second, what="", X=None, C=None, I=None):
    """Assignments equal the oracle's except where the oracle's relative gap
    between second-best and best is below TIE_GAP; there the GPU's block must
    itself be a near-best one: eff(p, A_gpu[p]) <= best*(1 + TIE_GAP).  The
    second check needs the points X, centers C and influence I."""
    A_gpu = np.asarray(A_gpu)
    k = len(I) if I is not None else None
    if k is not None:
        assert A_gpu.min(initial=0) >= 0 and A_gpu.max(initial=0) < k, f"{what}: block id out of range"
    bad = np.flatnonzero(A_gpu != A_orc)
    if bad.size:
        gap = (second[bad] - best[bad]) / np.maximum(best[bad], 1e-300)
        worst = float(gap.max())
        assert worst < TIE_GAP, (
            f"{what}: {bad.size} assignments differ, largest oracle gap {worst:.3e} "
            f"(first index {bad[0]}: gpu {A_gpu[bad[0]]} oracle {A_orc[bad[0]]})")
        if X is not None:
            e = effective_distance([np.asarray(x)[bad] for x in X], C, I, A_gpu[bad])
            assert np.all(e <= best[bad] * (1.0 + TIE_GAP)), (
                f"{what}: a differing GPU block is not within {TIE_GAP} of the best")
    return bad.size


def assert_centers_close(C_gpu, C_orc, X, what=""):
    ext = max(float(np.max(x) - np.min(x)) for x in X)
    scale = max(float(np.max(np.abs(C_orc))), ext)
    err = float(np.max(np.abs(np.asarray(C_gpu) - C_orc)))
    assert err <= CENTER_RTOL * scale, f"{what}: center error {err:.3e} > {CENTER_RTOL}*{scale:.3e}"
    return err
