"""Non-uniform target block sizes (the footnote to the objective at the
start of Sec. 4): every block has its own target weight and limit, and the
initial centers sit in proportion to the targets along the curve.  GPU runs
must equal the oracle's runs; equal targets must give the plain run."""
import numpy as np
import pytest

import oracle
from gpu_common import assert_centers_close, cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def _run_both(X, k, eps, t, W=None, max_iter=15, max_balance_iter=20, **kw):
    from paper_1805_01208_amd import bkm
    Xw = widened(X)
    Wd = None if W is None else torch.from_numpy(W).cuda()
    g = bkm.balanced_kmeans(cuda(X), k, W=Wd, eps=eps, max_iter=max_iter,
                            max_balance_iter=max_balance_iter,
                            target_sizes=torch.from_numpy(t).cuda(), **kw)
    o = oracle.balanced_kmeans(Xw, k, eps, W=W, max_iter=max_iter,
                               max_balance_iter=max_balance_iter, target_sizes=t)
    assert np.array_equal(g["A"].cpu().numpy(), o["A"])
    assert_centers_close(g["centers"].cpu().numpy(), o["centers"], Xw)
    gi, oi = g["info"], o["info"]
    assert (gi["rounds"], gi["sweeps"], gi["balanced"]) == (oi["rounds"], oi["sweeps"], oi["balanced"])
    if W is None:
        assert gi["l_max"] == oi["lmax"]
        assert gi["imbalance"] == oi["imbalance"]
    else:
        # node-weight totals: exact fixed-point sum against compensated summation
        assert gi["l_max"] == pytest.approx(oi["lmax"], rel=1e-13)
        assert gi["imbalance"] == pytest.approx(oi["imbalance"], rel=1e-12, abs=1e-13)
    return g, o


@pytest.mark.parametrize("precision", ["f32_recheck", "f64"])
def test_uniform_2d_matches_oracle(precision):
    print(f"case targets uniform 2D n=20000 k=6 {precision}", flush=True)
    X = workloads.uniform(20000, 2, 21)
    t = np.array([1.0, 2.0, 3.0, 4.0, 1.5, 0.5])
    g, _ = _run_both(X, 6, 0.05, t, max_iter=40, precision=precision)
    assert g["info"]["balanced"] == 1


def test_weighted_3d_matches_oracle():
    print("case targets weighted gauss 3D n=12000 k=16", flush=True)
    X = workloads.gauss3d(12000, 22)
    rng = np.random.default_rng(22)
    W = rng.lognormal(0.0, 0.5, 12000)
    t = rng.lognormal(0.0, 0.6, 16)
    _run_both(X, 16, 0.05, t, W=W, max_iter=20)


def test_f32_coordinates_many_blocks():
    print("case targets f32 refined 2D n=40000 k=64", flush=True)
    X = [x.astype(np.float32) for x in workloads.refined2d(40000, 23)]
    t = np.random.default_rng(23).uniform(0.2, 3.0, 64)
    _run_both(X, 64, 0.03, t, max_iter=12)


def test_more_blocks_than_one_prep_chunk():
    """k = 5000 target sizes: the prefix sums run over two LDS chunks."""
    print("case targets k=5000 n=20000 2D", flush=True)
    X = workloads.uniform(20000, 2, 24)
    t = np.random.default_rng(24).uniform(0.5, 1.5, 5000)
    _run_both(X, 5000, 0.1, t, max_iter=2, max_balance_iter=4)


def test_with_sample_init():
    from paper_1805_01208_amd import bkm
    print("case targets + sample init n=8000 3D k=8", flush=True)
    X = workloads.gauss3d(8000, 25)
    t = np.linspace(1.0, 3.0, 8)
    keys = workloads.splitmix64(25, 8000)
    g = bkm.balanced_kmeans(cuda(X), 8, eps=0.05, max_iter=20, sample_init=True,
                            sample_keys=torch.from_numpy(keys.view(np.int64)).cuda(),
                            target_sizes=torch.from_numpy(t).cuda())
    o = oracle.balanced_kmeans(X, 8, 0.05, max_iter=20, sample_keys=keys, target_sizes=t)
    assert np.array_equal(g["A"].cpu().numpy(), o["A"])
    assert g["info"]["sample_rounds"] == o["info"]["sample_rounds"]
    assert (g["info"]["rounds"], g["info"]["sweeps"]) == (o["info"]["rounds"], o["info"]["sweeps"])


def test_equal_targets_are_the_plain_run():
    from paper_1805_01208_amd import bkm
    print("case targets equal -> plain run, n=30000 k=24", flush=True)
    X = cuda(workloads.uniform(30000, 2, 26))
    g = bkm.balanced_kmeans(X, 24, max_iter=15, target_sizes=torch.full((24,), 2.0).cuda())
    h = bkm.balanced_kmeans(X, 24, max_iter=15)
    assert torch.equal(g["A"], h["A"]) and torch.equal(g["centers"], h["centers"])
    assert torch.equal(g["influence"], h["influence"])
    for key in ("rounds", "sweeps", "balanced", "l_max", "imbalance", "max_block_weight"):
        assert g["info"][key] == h["info"][key], key


@pytest.mark.parametrize("bad", [0.0, -2.0, float("nan"), float("inf")])
def test_invalid_target_sizes_are_rejected(bad):
    from paper_1805_01208_amd import bkm
    print(f"case targets invalid size {bad}", flush=True)
    X = cuda(workloads.uniform(2000, 2, 27))
    t = torch.ones(8, dtype=torch.float64)
    t[5] = bad
    with pytest.raises(bkm.BkmError, match="target_sizes"):
        bkm.balanced_kmeans(X, 8, target_sizes=t.cuda())
    with pytest.raises(bkm.BkmError, match="target_sizes"):
        bkm.partition_stats(X, torch.zeros(2000, dtype=torch.int32).cuda(), 8, target_sizes=t.cuda())
    with pytest.raises(bkm.BkmError, match="instance 1: target_sizes"):
        bkm.balanced_kmeans_batched([(X, 8), (X, 8)], target_sizes=[None, t.cuda()])


def test_partition_stats_with_targets():
    from paper_1805_01208_amd import bkm
    print("case targets stats n=9000 k=5", flush=True)
    X = workloads.uniform(9000, 2, 28)
    rng = np.random.default_rng(28)
    A = rng.integers(0, 5, 9000).astype(np.int32)
    t = np.array([1.0, 1.0, 2.0, 0.5, 4.0])
    for W in (None, rng.lognormal(0.0, 0.5, 9000)):
        Wd = None if W is None else torch.from_numpy(W).cuda()
        g = bkm.partition_stats(cuda(X), torch.from_numpy(A).cuda(), 5, 0.03, W=Wd,
                                target_sizes=torch.from_numpy(t).cuda())
        o = oracle.partition_stats(X, A, 5, 0.03, W=W, target_sizes=t)
        assert g["overloaded_blocks"] == o["overloaded_blocks"] >= 1
        assert g["l_max"] == pytest.approx(o["lmax"], rel=1e-13)
        assert g["imbalance"] == pytest.approx(o["imbalance"], rel=1e-12)


def test_batched_with_targets_matches_single_runs():
    from paper_1805_01208_amd import bkm
    print("case targets batched: 4 instances", flush=True)
    rng = np.random.default_rng(29)
    insts = [(cuda(workloads.uniform(15000, 2, 30)), 12),
             (cuda(workloads.gauss3d(9000, 31)), 7),
             (cuda(workloads.uniform(5000, 2, 32)), 20),
             (cuda(workloads.gauss3d(7000, 33)), 9)]
    ts = [torch.from_numpy(rng.uniform(0.5, 2.0, 12)).cuda(), None,
          torch.from_numpy(rng.uniform(0.1, 1.0, 20)).cuda(), torch.full((9,), 3.0).cuda()]
    outs, rc = bkm.balanced_kmeans_batched(insts, max_iter=12, target_sizes=ts)
    for (X, k), t, res in zip(insts, ts, outs):
        g = bkm.balanced_kmeans(X, k, max_iter=12, target_sizes=t)
        assert torch.equal(res["A"], g["A"]) and torch.equal(res["centers"], g["centers"])
        for key in ("rounds", "sweeps", "balanced", "imbalance", "l_max"):
            assert res["info"][key] == g["info"][key], key
