"""Pins of the oracle's full balanced k-means (Alg. 2 around Alg. 1):
the eps = infinity special case is Lloyd's algorithm (checked against
scikit-learn), k = 1 is trivial, and a finished run satisfies the balance
constraint and the weighted-mean invariant."""
import math

import numpy as np
import pytest

import oracle
from paper_1805_01208_amd import workloads


@pytest.mark.parametrize("d,rounds", [(2, 1), (2, 6), (3, 4)])
def test_infinite_eps_is_lloyd(d, rounds):
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(10 + d)
    n, k = 6000, 12
    X = [rng.random(n) for _ in range(d)]
    C0 = rng.random((k, d))
    r = oracle.balanced_kmeans(X, k, math.inf, max_iter=rounds, delta_threshold=0.0,
                               centers_init=C0)
    assert np.all(r["influence"] == 1.0)
    assert np.all(r["sweeps_per_round"] == 1)
    km = KMeans(n_clusters=k, init=C0, n_init=1, max_iter=rounds, tol=0.0,
                algorithm="lloyd").fit(np.stack(X, axis=1))
    assert np.allclose(r["centers"], km.cluster_centers_, rtol=0, atol=1e-12)


def test_single_block():
    rng = np.random.default_rng(3)
    n = 2000
    X = [rng.random(n), rng.random(n), rng.random(n)]
    W = rng.lognormal(0.0, 0.5, n)
    r = oracle.balanced_kmeans(X, 1, 0.03, W=W)
    assert np.all(r["A"] == 0)
    assert r["info"]["balanced"] == 1 and r["info"]["converged"] == 1
    assert r["info"]["rounds"] == 2  # second movement is exactly zero
    for j in range(3):
        assert r["centers"][0, j] == pytest.approx(math.fsum(W * X[j]) / math.fsum(W),
                                                   rel=1e-15)


def _check_means(X, W, A, C):
    k, d = C.shape
    w = np.ones(len(A)) if W is None else W
    for c in range(k):
        m = A == c
        if not m.any():
            continue
        for j in range(d):
            want = math.fsum(w[m] * X[j][m]) / math.fsum(w[m])
            assert C[c, j] == pytest.approx(want, rel=1e-14, abs=1e-15)


def test_c1_small_is_balanced_and_centers_are_means():
    cfg = workloads.c1(n=20000)
    r = oracle.balanced_kmeans(cfg["X"], cfg["k"], cfg["eps"])
    info = r["info"]
    assert info["balanced"] == 1
    assert r["block_weights"].max() <= info["lmax"]
    assert np.array_equal(r["block_weights"],
                          np.bincount(r["A"], minlength=cfg["k"]).astype(float))
    assert info["sweeps"] == r["sweeps_per_round"].sum()
    _check_means(cfg["X"], None, r["A"], r["centers"])


def test_weighted_3d_is_balanced():
    rng = np.random.default_rng(8)
    n, k = 20000, 24
    X = workloads.gauss3d(n, 8)
    W = rng.lognormal(0.0, 0.5, n)
    r = oracle.balanced_kmeans(X, k, 0.05, W=W, max_iter=30)
    assert r["info"]["balanced"] == 1
    assert r["block_weights"].max() <= r["info"]["lmax"]
    _check_means(X, W, r["A"], r["centers"])


def test_influence_balances_a_skewed_cloud():
    """Plain Voronoi cells of SFC-chosen centers on a clustered cloud are far
    from balanced; the influence update must bring them within L_max."""
    X = workloads.refined2d(30000, 2)
    k = 32
    r0 = oracle.balanced_kmeans(X, k, math.inf, max_iter=5)
    r = oracle.balanced_kmeans(X, k, 0.03, max_iter=50)
    lmax = oracle.lmax(30000, k, 0.03)
    assert r0["block_weights"].max() > lmax
    assert r["info"]["balanced"] == 1 and r["block_weights"].max() <= lmax
