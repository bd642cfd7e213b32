"""The sweep's autotuner: measured choices, the cache, and results that do
not depend on the tiling."""
import numpy as np
import pytest

import oracle
from gpu_common import cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def test_autotune_measures_then_caches():
    from paper_1805_01208_amd import bkm
    X = cuda(workloads.gauss3d(300000, 81))
    bkm.autotune_clear()
    print("case autotune measure + cache", flush=True)
    first = bkm.autotune(X, 60)
    assert first["from_cache"] == 0 and first["candidates"] == 12
    assert first["tile_points"] in (256, 512, 1024) and first["super_tiles"] in (8, 16, 24, 32)
    assert 0 < first["best_us"] <= first["default_us"]
    assert first["sample_points"] == 300000 and first["sample_k"] == 60
    again = bkm.autotune(X, 60)
    assert again["from_cache"] == 1
    assert (again["tile_points"], again["super_tiles"]) == (first["tile_points"], first["super_tiles"])
    # an explicit super-tile count is kept
    fixed = bkm.autotune(X, 60, super_tiles=5)
    assert fixed["super_tiles"] == 5 and fixed["from_cache"] == 1


def test_autotune_samples_large_inputs():
    """Above 2^23 points the tuner works on a strided sample with k scaled to
    keep the mean block size."""
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(82)
    n = 9_000_001
    X = [torch.from_numpy(rng.random(n, dtype=np.float32)).cuda() for _ in range(2)]
    print("case autotune sample", flush=True)
    r = bkm.autotune(X, 900, force=True)
    assert r["from_cache"] == 0 and r["sample_points"] == 4_500_001
    assert r["sample_k"] == 450


@pytest.mark.parametrize("precision", ["f64", "f32_recheck"])
def test_tuned_runs_equal_fixed_tile_runs_and_oracle(precision):
    """A run on the tuned tiling (fresh, then cached) gives the same
    assignment as runs on every fixed tile size, and the oracle's."""
    from paper_1805_01208_amd import bkm
    X = workloads.refined2d(60000, 83)
    Xd = cuda(X)
    k = 40
    bkm.autotune_clear()
    print(f"case tuned vs fixed {precision}", flush=True)
    fresh = bkm.balanced_kmeans(Xd, k, precision=precision, max_iter=15)
    cached = bkm.balanced_kmeans(Xd, k, precision=precision, max_iter=15)
    A = fresh["A"].cpu().numpy()
    assert np.array_equal(cached["A"].cpu().numpy(), A)
    for tile in (256, 512, 1024):
        for sup in (8, 32):
            g = bkm.balanced_kmeans(Xd, k, precision=precision, max_iter=15, tile_points=tile,
                                    super_tiles=sup)
            assert np.array_equal(g["A"].cpu().numpy(), A), (tile, sup)
    o = oracle.balanced_kmeans(widened(X), k, 0.03, max_iter=15)
    assert np.array_equal(A, o["A"])


def test_batched_call_uses_the_tuner():
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(84)
    insts = [(cuda(workloads.uniform(int(n), 2, 85 + i)), int(k))
             for i, (n, k) in enumerate([(20000, 8), (50000, 30), (35000, 12)])]
    bkm.autotune_clear()
    print("case batched autotune", flush=True)
    outs, rc = bkm.balanced_kmeans_batched(insts, max_iter=10, tile_points=0)
    assert rc in (0, 1)
    for (X, k), o in zip(insts, outs):
        assert bkm.autotune(X, k)["from_cache"] == 1
        g = bkm.balanced_kmeans(X, k, max_iter=10, tile_points=256)
        assert np.array_equal(o["A"].cpu().numpy(), g["A"].cpu().numpy())
