"""Pins of the oracle's non-uniform target block sizes (the footnote to the
objective at the start of Sec. 4), readings N1-N4: closed forms by hand,
the uniform special case, exact center positions, scale invariance, and the
balance definition met at the end of a run."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1805_01208_amd import workloads


def test_targets_closed_forms():
    # unit weights: n = 10, t = (1, 2, 7): T = 10 t / 10, L = 1.1 ceil(10 t / 10)
    T, L = oracle.targets(10, 3, 0.1, target_sizes=[1.0, 2.0, 7.0])
    assert list(T) == [1.0, 2.0, 7.0]
    assert list(L) == [1.1 * 1.0, 1.1 * 2.0, 1.1 * 7.0]
    # ceil of a fractional share: n = 10, t = (1, 1, 2) -> shares 2.5, 2.5, 5
    T, L = oracle.targets(10, 3, 0.0, target_sizes=[1.0, 1.0, 2.0])
    assert list(T) == [2.5, 2.5, 5.0] and list(L) == [3.0, 3.0, 5.0]
    # node weights summing to 20: T = 20 t / 4, L = (1 + eps) T
    W = np.array([4.0, 6.0, 2.5, 7.5])
    T, L = oracle.targets(4, 2, 0.5, W=W, target_sizes=[1.0, 3.0])
    assert list(T) == [5.0, 15.0] and list(L) == [7.5, 22.5]


def test_equal_targets_are_the_uniform_limits():
    for n, k, eps in ((10, 3, 0.1), (1000, 7, 0.03), (99991, 64, 0.0)):
        for t in (1.0, 2.5, 0.375):   # sums exact in FP64
            T, L = oracle.targets(n, k, eps, target_sizes=np.full(k, t))
            assert np.all(L == oracle.lmax(n, k, eps))
            assert np.all(T == n / k)


@pytest.mark.parametrize("bad", [0.0, -1.0, math.nan, math.inf])
def test_invalid_target_sizes_are_rejected(bad):
    with pytest.raises(RuntimeError):
        oracle.targets(10, 2, 0.1, target_sizes=[1.0, bad])


def test_balance_step_per_block():
    # block 1 exceeds its own limit although block 0 is larger
    s = np.array([25.0, 8.0])
    ok, I = oracle.balance_step_targets(s, 2, [26.0, 6.0], [25.0, 5.0], [1.0, 1.0])
    assert not ok
    assert I[0] == 1.0                      # sqrt(25/25)
    assert I[1] == 0.95                     # sqrt(5/8) = 0.79 -> clamp
    # every block within its own limit: balanced, influence untouched
    ok, I = oracle.balance_step_targets([25.0, 5.0], 3, [26.0, 6.0], [25.0, 5.0], [2.0, 3.0])
    assert ok and list(I) == [2.0, 3.0]
    # closed form inside the clamp, d = 3, and an empty block
    ok, I = oracle.balance_step_targets([10.0, 0.0, 12.0], 3, [10.5, 1.0, 10.5],
                                        [10.0, 1.0, 11.0], [1.0, 1.0, 1.0])
    assert not ok
    assert I[0] == 1.0 and I[1] == 1.05 and I[2] == pytest.approx((11.0 / 12.0) ** (1 / 3), rel=1e-15)


def test_balance_step_with_constant_targets_is_the_uniform_step():
    rng = np.random.default_rng(3)
    for _ in range(20):
        k = int(rng.integers(2, 30))
        s = rng.integers(0, 50, k).astype(np.float64)
        I0 = rng.uniform(0.5, 2.0, k)
        lm, T = float(rng.uniform(20, 40)), float(rng.uniform(10, 30))
        a = oracle.balance_step(s, 2, lm, T, I0)
        b = oracle.balance_step_targets(s, 2, np.full(k, lm), np.full(k, T), I0)
        assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_initial_centers_in_proportion_to_targets():
    """Center c sits at sorted position floor(n S_c / tsum) + floor(n t_c / (2 tsum)),
    evaluated here in exact rationals (every quotient that is an integer is
    exactly representable, so the FP64 floors agree)."""
    X = workloads.uniform(1000, 2, 8)
    t = [1.0, 2.0, 3.0, 4.0, 5.0]
    C, perm, keys = oracle.init_centers_sfc(X, 5, 16, target_sizes=t)
    order = np.lexsort((np.arange(1000), keys))
    n, tsum = 1000, Fraction(15)
    S = Fraction(0)
    for c, tc in enumerate(t):
        pos = math.floor(n * S / tsum) + math.floor(n * Fraction(tc) / (2 * tsum))
        assert list(C[c]) == [X[0][order[pos]], X[1][order[pos]]]
        S += Fraction(tc)
    # the last position is clamped to n - 1
    C2, _, _ = oracle.init_centers_sfc(X[:2], 2, 16, target_sizes=[1.0, 1e-300])
    assert list(C2[1]) == [X[0][order[-1]], X[1][order[-1]]]
    # equal targets: the evenly spaced positions
    Cu, _, _ = oracle.init_centers_sfc(X, 7, 16, target_sizes=np.full(7, 0.375))
    C0, _, _ = oracle.init_centers_sfc(X, 7, 16)
    assert np.array_equal(Cu, C0)


def test_equal_targets_reproduce_the_plain_run():
    cfg = workloads.c1(n=6000)
    W = np.random.default_rng(4).lognormal(0.0, 0.5, 6000)
    for w in (None, W):
        a = oracle.balanced_kmeans(cfg["X"], 12, 0.03, W=w, max_iter=15, target_sizes=np.full(12, 3.0))
        b = oracle.balanced_kmeans(cfg["X"], 12, 0.03, W=w, max_iter=15)
        assert np.array_equal(a["A"], b["A"])
        assert np.array_equal(a["centers"], b["centers"])
        assert np.array_equal(a["influence"], b["influence"])
        assert a["info"] == b["info"]


def test_scaling_the_targets_by_a_power_of_two_changes_nothing():
    X = workloads.gauss3d(5000, 9)
    t = np.random.default_rng(9).uniform(0.5, 2.0, 10)
    a = oracle.balanced_kmeans(X, 10, 0.05, max_iter=10, target_sizes=t)
    b = oracle.balanced_kmeans(X, 10, 0.05, max_iter=10, target_sizes=4.0 * t)
    assert np.array_equal(a["A"], b["A"]) and np.array_equal(a["centers"], b["centers"])


def test_infinite_eps_with_targets_is_lloyd_from_the_target_positions():
    from sklearn.cluster import KMeans
    X = workloads.uniform(3000, 2, 10)
    t = [1.0, 3.0, 2.0, 6.0]
    r = oracle.balanced_kmeans(X, 4, math.inf, max_iter=3, delta_threshold=0.0, target_sizes=t)
    C0, _, _ = oracle.init_centers_sfc(X, 4, 16, target_sizes=t)
    P = np.stack(X, axis=1)
    km = KMeans(n_clusters=4, init=C0, n_init=1, max_iter=3, tol=0.0, algorithm="lloyd").fit(P)
    assert np.allclose(r["centers"], km.cluster_centers_, rtol=0, atol=1e-12)
    assert np.all(r["influence"] == 1.0)


@pytest.mark.parametrize("weighted", [False, True])
def test_run_meets_each_blocks_limit(weighted):
    rng = np.random.default_rng(11)
    n, k = 20000, 6
    X = workloads.uniform(n, 2, 12)
    W = rng.lognormal(0.0, 0.4, n) if weighted else None
    t = np.array([1.0, 2.0, 3.0, 4.0, 1.5, 0.5])
    r = oracle.balanced_kmeans(X, k, 0.05, W=W, max_iter=60, target_sizes=t)
    w = np.ones(n) if W is None else W
    s = np.bincount(r["A"], weights=w, minlength=k)
    wt = math.fsum(w)
    T = wt * t / t.sum()
    L = 1.05 * (np.ceil(n * t / t.sum()) if W is None else T)
    assert r["info"]["balanced"] == 1
    assert np.all(s <= L)
    assert r["info"]["imbalance"] == pytest.approx(np.max(s / T) - 1.0, rel=1e-12)
    assert r["info"]["lmax"] == pytest.approx(L.max(), rel=1e-15)
    st = oracle.partition_stats(X, r["A"], k, 0.05, W=W, target_sizes=t)
    assert st["overloaded_blocks"] == 0
    assert st["imbalance"] == pytest.approx(np.max(s / T) - 1.0, rel=1e-12)
    # the same assignment against equal targets is badly overloaded
    su = oracle.partition_stats(X, r["A"], k, 0.05, W=W)
    assert su["overloaded_blocks"] >= 2


def test_sample_init_with_targets_ends_balanced():
    X = workloads.gauss3d(8000, 13)
    t = np.linspace(1.0, 3.0, 8)
    keys = workloads.splitmix64(21, 8000)
    r = oracle.balanced_kmeans(X, 8, 0.05, max_iter=40, sample_keys=keys, target_sizes=t)
    s = np.bincount(r["A"], minlength=8)
    assert r["info"]["balanced"] == 1
    assert np.all(s <= 1.05 * np.ceil(8000 * t / t.sum()))
