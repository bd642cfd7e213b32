"""Many balanced k-means runs in one call (Alg. 2 around Alg. 1 per instance):
each instance must come out exactly as a separate run with the same
parameters, and, where the oracle is fast enough, as the oracle's run."""
import numpy as np
import pytest

import oracle
from gpu_common import assert_centers_close, cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def _same_as_single(bkm, inst, res, **kw):
    X, k = inst[0], inst[1]
    W = inst[2] if len(inst) > 2 else None
    g = bkm.balanced_kmeans(X, k, W=W, **kw)
    assert torch.equal(res["A"], g["A"])
    assert torch.equal(res["centers"], g["centers"])
    for key in ("rounds", "sweeps", "balanced", "converged", "evaluated", "skipped", "changed"):
        assert res["info"][key] == g["info"][key], key


def test_mixed_batch_matches_single_runs_and_oracle():
    """2D and 3D, FP64 and FP32 coordinates, node weights, tiny and
    degenerate instances, three tile sizes, in one call."""
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(77)
    specs = [
        (workloads.uniform(20000, 2, 1), 16, None),
        (workloads.gauss3d(15000, 2), 24, None),
        ([x.astype(np.float32) for x in workloads.uniform(9000, 2, 3)], 40, None),
        (workloads.gauss3d(6000, 4), 9, rng.lognormal(0.0, 0.5, 6000)),
        (workloads.refined2d(30000, 5), 64, None),
        ([rng.random(5), rng.random(5)], 5, None),
        ([rng.random(300), rng.random(300), rng.random(300)], 1, None),
        (workloads.uniform(4000, 2, 6), 300, None),
    ]
    insts = []
    for X, k, W in specs:
        Xd = cuda(X)
        insts.append((Xd, k) if W is None else (Xd, k, torch.from_numpy(W).cuda()))
    tiles = [0, 1024, 512, 256, 0, 256, 0, 0]
    print(f"case batched mixed: {len(insts)} instances", flush=True)
    outs, rc = bkm.balanced_kmeans_batched(insts, max_iter=15, tile_points=tiles)
    assert rc in (0, 1)
    for i, ((X, k, W), inst, res) in enumerate(zip(specs, insts, outs)):
        print(f"  instance {i}: n={len(X[0])} d={len(X)} k={k}", flush=True)
        _same_as_single(bkm, inst, res, max_iter=15, tile_points=tiles[i])
        o = oracle.balanced_kmeans(widened(X), k, 0.03, W=W, max_iter=15)
        assert np.array_equal(res["A"].cpu().numpy(), o["A"]), f"instance {i}"
        assert_centers_close(res["centers"].cpu().numpy(), o["centers"], X, f"instance {i}")
        assert (res["info"]["rounds"], res["info"]["sweeps"]) == (o["info"]["rounds"],
                                                                  o["info"]["sweeps"])


def test_batch_recipe_scaled_down():
    """The batched workload's recipe (n and k log-uniform, even ids 2D
    uniform, odd ids 3D Gaussian clusters) at 48 instances of up to 40 000
    points, both precisions, against separate runs."""
    from paper_1805_01208_amd import bkm
    cfgs = workloads.c4(count=48, n_lo=2000, n_hi=40000, k_lo=4, k_hi=256)
    insts = [(cuda(c["X"]), c["k"]) for c in cfgs]
    for prec in ("f32_recheck", "f64"):
        print(f"case batched recipe: {len(insts)} instances {prec}", flush=True)
        outs, rc = bkm.balanced_kmeans_batched(insts, max_iter=10, precision=prec)
        assert rc in (0, 1)
        for i in range(0, len(insts), 5):
            _same_as_single(bkm, insts[i], outs[i], max_iter=10, precision=prec)
        # a few against the oracle
        for i in (0, 1, 2, 3):
            c = cfgs[i]
            o = oracle.balanced_kmeans(widened(c["X"]), c["k"], 0.03, max_iter=10)
            assert np.array_equal(outs[i]["A"].cpu().numpy(), o["A"]), f"instance {i}"


def test_batch_of_one_equals_single_call():
    from paper_1805_01208_amd import bkm
    cfg = workloads.c1(n=30000)
    inst = (cuda(cfg["X"]), cfg["k"])
    outs, rc = bkm.balanced_kmeans_batched([inst])
    _same_as_single(bkm, inst, outs[0])
    assert outs[0]["info"]["balanced"] == 1 and rc == 0


def test_batched_data_error_names_instance():
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(3)
    good = [rng.random(1000), rng.random(1000)]
    bad = [rng.random(1000), rng.random(1000)]
    bad[1][17] = np.nan
    with pytest.raises(bkm.BkmError, match="instance 1"):
        bkm.balanced_kmeans_batched([(cuda(good), 8), (cuda(bad), 8)])
