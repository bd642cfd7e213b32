"""The device debug mode: after every sweep and every center move, sampled
(or all) points are checked in exact FP64 against every center -- stored
Hamerly bounds valid (Sec. 4.3; Eqs. 2-3 read as relaxations), block an
argmin after a sweep.  Runs with the checks must report no violation and
give the same result as runs without them."""
import numpy as np
import pytest

from gpu_common import cuda, torch
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu

CASES = [
    ("uniform2d", lambda: workloads.uniform(40000, 2, 91), 24, {}),
    ("gauss3d", lambda: workloads.gauss3d(50000, 92), 40, {"eps": 0.01}),
    ("refined2d-f64", lambda: workloads.refined2d(60000, 93), 64, {"precision": "f64"}),
    ("gauss3d-no-erosion", lambda: workloads.gauss3d(30000, 94), 16, {"erosion": False}),
    ("uniform2d-sample-start", lambda: workloads.uniform(80000, 2, 95), 8,
     {"sample_init": True, "seed": 3}),
]


@pytest.mark.parametrize("name,make,k,kw", CASES, ids=[c[0] for c in CASES])
def test_debug_checks_every_point(name, make, k, kw):
    from paper_1805_01208_amd import bkm
    X = cuda(make())
    print(f"case debug checks {name}", flush=True)
    ref = bkm.balanced_kmeans(X, k, max_iter=20, **kw)
    g = bkm.balanced_kmeans(X, k, max_iter=20, debug_checks=2, **kw)
    info = g["info"]
    n = X[0].numel()
    # every point, after every sweep and every move
    assert info["debug_checked"] >= n * info["sweeps"]
    assert info["debug_violations"] == 0
    assert torch.equal(g["A"], ref["A"]) and torch.equal(g["centers"], ref["centers"])


def test_debug_checks_weighted_and_targets():
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(96)
    X = cuda(workloads.gauss3d(40000, 97))
    W = torch.from_numpy(rng.lognormal(0.0, 0.5, 40000)).cuda()
    t = torch.from_numpy(rng.uniform(0.5, 2.0, 30)).cuda()
    print("case debug checks weighted + targets", flush=True)
    g = bkm.balanced_kmeans(X, 30, W=W, target_sizes=t, max_iter=20, debug_checks=2)
    assert g["info"]["debug_checked"] > 0 and g["info"]["debug_violations"] == 0


def test_debug_checks_sampled_on_a_large_cloud():
    """Mode 1 samples about 2^26 point-center pairs per check."""
    from paper_1805_01208_amd import bkm
    X = cuda(workloads.c3(n=2_000_000, k=128)["X"])
    print("case debug checks sampled 2M 3D", flush=True)
    g = bkm.balanced_kmeans(X, 128, max_iter=10, debug_checks=1)
    info = g["info"]
    assert 0 < info["debug_checked"] < 2_000_000 * info["sweeps"]
    assert info["debug_violations"] == 0
