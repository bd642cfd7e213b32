"""Random-sample initialization (the random start described with Alg. 2):
rounds on nested random samples doubling from a first sample (by default
100 points per block), then the main
loop on all points.  The GPU run must equal the oracle's run with the same
random order keys, and its own splitmix64 keys must be the published
generator's."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import assert_centers_close, cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def _keys_dev(keys):
    return torch.from_numpy(keys.view(np.int64)).cuda()


def _check_against_oracle(X, k, eps, W=None, max_iter=12, seed=0, start=100, **kw):
    from paper_1805_01208_amd import bkm
    Xw = widened(X)
    n = len(Xw[0])
    keys = workloads.splitmix64(seed, n)
    Wd = None if W is None else torch.from_numpy(W).cuda()
    g = bkm.balanced_kmeans(cuda(X), k, W=Wd, eps=eps, max_iter=max_iter, sample_init=True,
                            sample_start=start, sample_keys=_keys_dev(keys), **kw)
    o = oracle.balanced_kmeans(Xw, k, eps, W=W, max_iter=max_iter, sample_keys=keys,
                               sample_start=start)
    assert np.array_equal(g["A"].cpu().numpy(), o["A"])
    assert_centers_close(g["centers"].cpu().numpy(), o["centers"], Xw)
    gi, oi = g["info"], o["info"]
    assert (gi["sample_rounds"], gi["sample_sweeps"]) == (oi["sample_rounds"], oi["sample_sweeps"])
    assert (gi["rounds"], gi["sweeps"]) == (oi["rounds"], oi["sweeps"])
    assert gi["balanced"] == oi["balanced"]
    s0 = start if start > 0 else 100 * k
    assert gi["sample_rounds"] == (math.ceil(math.log2(n / s0)) if n > s0 else 0)
    return g


@pytest.mark.parametrize("precision", ["f32_recheck", "f64"])
def test_uniform_2d_matches_oracle(precision):
    print(f"case sample-init uniform 2D n=20000 k=16 {precision}", flush=True)
    X = workloads.uniform(20000, 2, 11)
    _check_against_oracle(X, 16, 0.03, seed=5, precision=precision)


def test_weighted_gauss_3d_matches_oracle():
    print("case sample-init weighted gauss 3D n=8000 k=12", flush=True)
    X = workloads.gauss3d(8000, 12)
    W = np.random.default_rng(12).lognormal(0.0, 0.5, 8000)
    _check_against_oracle(X, 12, 0.05, W=W, seed=7)


def test_f32_coordinates_match_oracle():
    print("case sample-init f32 refined 2D n=30000 k=40", flush=True)
    X = [x.astype(np.float32) for x in workloads.refined2d(30000, 13)]
    _check_against_oracle(X, 40, 0.03, seed=8)


def test_more_blocks_than_first_sample():
    """k = 300 centers against a first sample of 100 points."""
    print("case sample-init k=300 > 100 sample points, n=4000", flush=True)
    X = workloads.uniform(4000, 2, 14)
    _check_against_oracle(X, 300, 0.05, seed=9, max_iter=10)


def test_odd_start_and_tiles():
    print("case sample-init start=37, tile 256, n=5000 3D k=20", flush=True)
    X = workloads.gauss3d(5000, 15)
    _check_against_oracle(X, 20, 0.03, seed=10, start=37, tile_points=256)


def test_sample_start_of_one_point():
    """sample_start = 1: the first rounds run on 1, 2, 4, ... points with
    all k centers (most blocks empty)."""
    print("case sample-init start=1, n=300 2D k=8", flush=True)
    X = workloads.uniform(300, 2, 18)
    _check_against_oracle(X, 8, 0.05, seed=11, start=1, max_iter=8)


def test_default_keys_are_splitmix64():
    """Without caller keys the library draws splitmix64(seed, i) itself: the
    run must equal the one given those keys explicitly."""
    from paper_1805_01208_amd import bkm
    print("case sample-init generated keys, n=12000 k=24", flush=True)
    X = cuda(workloads.uniform(12000, 2, 16))
    for seed in (0, 123456789, 2**64 - 1):
        g = bkm.balanced_kmeans(X, 24, max_iter=8, sample_init=True, seed=seed)
        h = bkm.balanced_kmeans(X, 24, max_iter=8, sample_init=True,
                                sample_keys=_keys_dev(workloads.splitmix64(seed, 12000)))
        assert torch.equal(g["A"], h["A"]) and torch.equal(g["centers"], h["centers"])
        assert g["info"]["sample_rounds"] == 3   # from 100 * 24 points: 2400, 4800, 9600


def test_default_start_is_100_points_per_block():
    """sample_start = 0 (the default): the first sample has 100 * k points,
    as the oracle reads it too."""
    print("case sample-init default start, n=40000 2D k=25", flush=True)
    X = workloads.refined2d(40000, 19)
    g = _check_against_oracle(X, 25, 0.03, seed=12, start=0, max_iter=10)
    assert g["info"]["sample_rounds"] == 4   # 2500, 5000, 10000, 20000


def test_sample_covering_all_points_is_plain_run():
    from paper_1805_01208_amd import bkm
    print("case sample-init start >= n, n=3000 k=8", flush=True)
    X = cuda(workloads.uniform(3000, 2, 17))
    g = bkm.balanced_kmeans(X, 8, max_iter=10, sample_init=True, sample_start=3000)
    h = bkm.balanced_kmeans(X, 8, max_iter=10)
    assert torch.equal(g["A"], h["A"]) and torch.equal(g["centers"], h["centers"])
    assert g["info"]["sample_rounds"] == 0 and g["info"]["sample_sweeps"] == 0
