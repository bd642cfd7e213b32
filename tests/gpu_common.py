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


def assert_assignment_parity(A_gpu, A_orc, best, second, what=""):
    A_gpu = np.asarray(A_gpu)
    bad = np.flatnonzero(A_gpu != A_orc)
    if bad.size:
        gap = (second[bad] - best[bad]) / np.maximum(best[bad], 1e-300)
        worst = float(gap.max())
        assert worst < TIE_GAP, (
            f"{what}: {bad.size} assignments differ, largest oracle gap {worst:.3e} "
            f"(first index {bad[0]}: gpu {A_gpu[bad[0]]} oracle {A_orc[bad[0]]})")
    return bad.size


def assert_centers_close(C_gpu, C_orc, X, what=""):
    ext = max(float(np.max(x) - np.min(x)) for x in X)
    scale = max(float(np.max(np.abs(C_orc))), ext)
    err = float(np.max(np.abs(np.asarray(C_gpu) - C_orc)))
    assert err <= CENTER_RTOL * scale, f"{what}: center error {err:.3e} > {CENTER_RTOL}*{scale:.3e}"
    return err
