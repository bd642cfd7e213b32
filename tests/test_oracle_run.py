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


# ---------------------------------------------------------------- random-sample initialization
def test_sample_init_with_eps_infinite_is_lloyd_on_nested_samples():
    """With eps = infinity every AssignAndBalance call balances at its first
    sweep and the influence stays 1, so the random-sample initialization is
    one Lloyd step on each nested sample (the first s points of the random
    order, s = 100, 200, ...) followed by the run on all points; checked
    against scikit-learn's Lloyd steps from the same SFC centers."""
    from sklearn.cluster import KMeans
    rng = np.random.default_rng(31)
    n, k = 2000, 4
    X = [rng.random(n), rng.random(n)]
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    r = oracle.balanced_kmeans(X, k, math.inf, max_iter=1, delta_threshold=0.0,
                               sample_keys=keys, sample_start=100)
    assert r["info"]["sample_rounds"] == math.ceil(math.log2(n / 100))
    assert np.all(r["influence"] == 1.0)
    order = np.lexsort((np.arange(n), keys))        # by key, then index
    P = np.stack(X, axis=1)
    C, _, _ = oracle.init_centers_sfc(X, k, 16)
    s = 100
    while s < n:
        C = KMeans(n_clusters=k, init=C, n_init=1, max_iter=1, tol=0.0,
                   algorithm="lloyd").fit(P[order[:s]]).cluster_centers_
        s *= 2
    C = KMeans(n_clusters=k, init=C, n_init=1, max_iter=1, tol=0.0,
               algorithm="lloyd").fit(P).cluster_centers_
    assert np.allclose(r["centers"], C, rtol=0, atol=1e-12)


def test_sample_init_with_one_sample_covering_everything_is_the_plain_run():
    cfg = workloads.c1(n=90)
    keys = np.arange(90, dtype=np.uint64)[::-1].copy()
    a = oracle.balanced_kmeans(cfg["X"], 6, 0.03, max_iter=8, sample_keys=keys, sample_start=100)
    b = oracle.balanced_kmeans(cfg["X"], 6, 0.03, max_iter=8)
    assert a["info"]["sample_rounds"] == 0
    assert np.array_equal(a["A"], b["A"])
    assert np.array_equal(a["centers"], b["centers"])
    assert np.array_equal(a["influence"], b["influence"])


def test_sample_init_finishes_balanced_with_block_means():
    """A weighted 3D run with the random-sample start still ends balanced,
    with centers the weighted means."""
    rng = np.random.default_rng(33)
    n, k = 8000, 40
    X = [rng.random(n) for _ in range(3)]
    W = rng.lognormal(0.0, 0.5, n)
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    r = oracle.balanced_kmeans(X, k, 0.05, W=W, max_iter=30, sample_keys=keys, sample_start=100)
    assert r["info"]["sample_rounds"] == math.ceil(math.log2(n / 100))
    assert r["info"]["balanced"] == 1
    assert r["block_weights"].max() <= r["info"]["lmax"]
    _check_means(X, W, r["A"], r["centers"])


def test_sample_rounds_with_more_blocks_than_sample_points():
    """k = 300 > the first sample of 100 points: the sample rounds run with
    empty blocks (they keep their centers and gain influence) and the run
    on all points still ends with centers the means of their blocks."""
    rng = np.random.default_rng(34)
    n, k = 6000, 300
    X = [rng.random(n), rng.random(n)]
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    r = oracle.balanced_kmeans(X, k, 0.05, max_iter=10, sample_keys=keys, sample_start=100)
    assert r["info"]["sample_rounds"] == math.ceil(math.log2(n / 100))
    _check_means(X, None, r["A"], r["centers"])


def test_default_first_sample_is_100_points_per_block():
    """sample_start = 0 (the default) starts from 100 points per block,
    100 * k: the paper starts every process with 100 of its points and runs
    one block per process, so the number of sample rounds is
    ceil(log2(n_local / 100)) with n_local = n / k."""
    rng = np.random.default_rng(35)
    n, k = 20000, 16
    X = [rng.random(n), rng.random(n)]
    keys = rng.integers(0, 2**63, n, dtype=np.uint64)
    a = oracle.balanced_kmeans(X, k, 0.03, max_iter=8, sample_keys=keys)
    b = oracle.balanced_kmeans(X, k, 0.03, max_iter=8, sample_keys=keys, sample_start=100 * k)
    assert a["info"]["sample_rounds"] == math.ceil(math.log2((n / k) / 100)) == 4
    assert a["info"]["sample_rounds"] == b["info"]["sample_rounds"]
    assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["centers"], b["centers"])
    # n <= 100 k: no sample round at all
    c = oracle.balanced_kmeans(X, 200, 0.03, max_iter=3, sample_keys=keys)
    assert c["info"]["sample_rounds"] == 0


def test_sample_init_is_the_composition_of_single_rounds():
    """The sampled run equals single one-round runs on the nested samples
    (first 100, 200, ... points in (key, index) order), each starting from
    the previous round's centers and influences, then the run on all points:
    the composition is redone here in Python around the pinned single run,
    with node weights and a finite eps so that the influences matter."""
    rng = np.random.default_rng(35)
    n, k = 1500, 5
    X = [rng.random(n), rng.random(n)]
    W = rng.lognormal(0.0, 0.5, n)
    keys = workloads.splitmix64(35, n)
    r = oracle.balanced_kmeans(X, k, 0.02, W=W, max_iter=6, sample_keys=keys, sample_start=100)
    order = np.lexsort((np.arange(n), keys))
    dthr = 1e-5 * max(float(x.max() - x.min()) for x in X)
    C, _, _ = oracle.init_centers_sfc(X, k, 16)
    I = np.ones(k)
    s = 100
    rounds = 0
    while s < n:
        idx = order[:s]
        o = oracle.balanced_kmeans([x[idx] for x in X], k, 0.02, W=W[idx], max_iter=1,
                                   delta_threshold=dthr, centers_init=C, influence_init=I)
        C, I = o["centers"], o["influence"]
        s *= 2
        rounds += 1
    assert not np.all(I == 1.0)          # the influences were carried, not reset
    full = oracle.balanced_kmeans(X, k, 0.02, W=W, max_iter=6, delta_threshold=dthr,
                                  centers_init=C, influence_init=I)
    assert r["info"]["sample_rounds"] == rounds == 4
    assert np.array_equal(r["A"], full["A"])
    assert np.array_equal(r["centers"], full["centers"])
    assert np.array_equal(r["influence"], full["influence"])


def test_erosion_off_is_the_loop_of_pinned_steps():
    """With erosion off, the run is the loop of the pinned single steps (Alg.
    2 around Alg. 1): assign, block weights, balance test and influence step,
    new centers, and nothing between rounds.  Redone here in Python around
    those steps; with erosion on, the influences differ."""
    rng = np.random.default_rng(36)
    n, k, eps = 3000, 7, 0.01
    X = [rng.random(n), rng.random(n)]
    dthr = 1e-5 * max(float(x.max() - x.min()) for x in X)
    r = oracle.balanced_kmeans(X, k, eps, max_iter=4, max_balance_iter=3, delta_threshold=dthr,
                               erosion=False)
    C, _, _ = oracle.init_centers_sfc(X, k, 16)
    I = np.ones(k)
    lm = oracle.lmax(n, k, eps)
    for _ in range(4):
        for _ in range(3):
            A, _, _ = oracle.assign(X, C, I)
            bw = oracle.block_weights(A, None, k)
            ok, I = oracle.balance_step(bw, 2, lm, n / k, I)
            if ok:
                break
        Cn, delta = oracle.new_centers(X, None, A, C)
        C = Cn
        if delta.max() < dthr:
            break
    assert np.array_equal(r["A"], A)
    assert np.array_equal(r["centers"], C)
    assert np.array_equal(r["influence"], I)
    e = oracle.balanced_kmeans(X, k, eps, max_iter=4, max_balance_iter=3, delta_threshold=dthr)
    assert not np.array_equal(e["influence"], I)


@pytest.mark.parametrize("weighted", [False, True])
def test_erosion_on_is_the_loop_of_pinned_steps(weighted):
    """With erosion on (the default of every run), the run is the loop of the
    pinned single steps with erosion placed as Sec. 4.2 and Alg. 2 read:
    AssignAndBalance, new centers; on convergence the new centers are
    returned as they are; otherwise beta is taken from the round's final
    assignment, the influence is eroded by the round's movements, and only
    then do the new centers replace the old ones.  Redone here in Python
    around those steps, for unit and node weights, bit for bit."""
    rng = np.random.default_rng(37 + weighted)
    n, k, eps, rounds, sweeps = 3000, 7, 0.01, 50, 3
    X = [rng.random(n), rng.random(n)]
    W = rng.lognormal(0.0, 0.5, n) if weighted else None
    # a threshold the run meets with a movement that is not zero, so that an
    # erosion on the converged round would change the returned influence
    dthr = 1e-3
    r = oracle.balanced_kmeans(X, k, eps, W=W, max_iter=rounds, max_balance_iter=sweeps,
                               delta_threshold=dthr)
    C, _, _ = oracle.init_centers_sfc(X, k, 16)
    I = np.ones(k)
    lm = oracle.lmax(n, k, eps, W)
    target = oracle.total_weight(n, W) / k
    eroded = made = 0
    for _ in range(rounds):
        made += 1
        for _ in range(sweeps):
            A, _, _ = oracle.assign(X, C, I)
            bw = oracle.block_weights(A, W, k)
            ok, I = oracle.balance_step(bw, 2, lm, target, I)
            if ok:
                break
        Cn, delta = oracle.new_centers(X, W, A, C)
        if delta.max() < dthr:
            assert delta.max() > 0.0
            C = Cn
            break
        I = oracle.erode(delta, oracle.beta(X, A, k), I)
        eroded += 1
        C = Cn
    assert eroded >= 2                       # erosion acted between rounds
    assert np.array_equal(r["A"], A)
    assert np.array_equal(r["centers"], C)
    assert np.array_equal(r["influence"], I)
    assert r["info"]["rounds"] == made < rounds
    assert r["info"]["converged"] == 1       # the last round returned without erosion
