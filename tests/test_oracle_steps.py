"""Pins of the oracle's per-step arithmetic: block weights (Alg. 1), balance
bound L_max (Sec. 2), influence adaptation with the 5% clamp (Sec. 4.2,
Eq. 1), weighted centers and movement (Alg. 2), beta and influence erosion
(Sec. 4.2), partition statistics."""
import math

import numpy as np
import pytest

import oracle


def test_block_weights_unit_is_bincount():
    rng = np.random.default_rng(1)
    A = rng.integers(0, 37, 100000).astype(np.int32)
    bw = oracle.block_weights(A, None, 40)
    assert np.array_equal(bw, np.bincount(A, minlength=40).astype(np.float64))


def test_block_weights_weighted_is_fsum():
    rng = np.random.default_rng(2)
    A = rng.integers(0, 9, 20000).astype(np.int32)
    W = rng.lognormal(0.0, 0.5, 20000)
    bw = oracle.block_weights(A, W, 10)
    for c in range(10):
        assert bw[c] == pytest.approx(math.fsum(W[A == c]), rel=2e-16, abs=0)
    assert bw[9] == 0.0


def test_lmax_closed_forms():
    # unit weights: (1 + eps) * ceil(n / k)
    assert oracle.lmax(100000, 16, 0.03) == 6437.5
    assert oracle.lmax(100001, 16, 0.0) == 6251.0
    # node weights: (1 + eps) * W / k
    W = np.full(10, 0.5)
    assert oracle.lmax(10, 4, 0.5, W) == pytest.approx(1.5 * 5.0 / 4)


def test_balanced_sizes_leave_influence_alone():
    sizes = np.array([100.0, 103.0, 97.0, 100.0])
    b, I = oracle.balance_step(sizes, 2, 103.0, 100.0, np.array([1.0, 2.0, 0.5, 1.1]))
    assert b and np.array_equal(I, [1.0, 2.0, 0.5, 1.1])


def test_influence_direction_and_magnitude():
    """Oversized blocks lose influence, undersized gain (Sec. 4.2 prose);
    unclamped the factor is (target/size)^(1/d), i.e. the new influence to the
    d-th power changes by target/size; the step is clamped to 5%; an empty
    block grows by 5%."""
    T = 100.0
    sizes = np.array([T / 1.0404, T * 1.0404, T / 1.030301, 0.0, 1e9, 1e-3 * T, T])
    I0 = np.array([1.0, 1.0, 2.0, 1.0, 1.0, 1.0, 3.0])
    b, I2 = oracle.balance_step(sizes, 2, 101.0, T, I0)
    assert not b
    assert I2[0] == pytest.approx(1.02, rel=1e-15)
    assert I2[1] == pytest.approx(1 / 1.02, rel=1e-15)
    assert I2[3] == pytest.approx(1.05, rel=1e-16)
    assert I2[4] == pytest.approx(0.95, rel=1e-16)
    assert I2[5] == pytest.approx(1.05, rel=1e-16)
    assert I2[6] == 3.0
    b, I3 = oracle.balance_step(sizes, 3, 101.0, T, I0)
    assert I3[2] == pytest.approx(2.0 * 1.01, rel=1e-15)
    assert (I3[0] / I0[0]) ** 3 == pytest.approx(1.0404, rel=1e-14)


def test_new_centers_are_weighted_means_and_delta():
    rng = np.random.default_rng(4)
    n, k = 5000, 6
    X = [rng.random(n), rng.random(n), rng.random(n)]
    W = rng.lognormal(0, 0.5, n)
    A = rng.integers(0, k - 1, n).astype(np.int32)  # block k-1 stays empty
    C0 = rng.random((k, 3))
    C1, delta = oracle.new_centers(X, W, A, C0)
    for c in range(k - 1):
        m = A == c
        for j in range(3):
            want = math.fsum(W[m] * X[j][m]) / math.fsum(W[m])
            assert C1[c, j] == pytest.approx(want, rel=1e-15, abs=1e-16)
        assert delta[c] == pytest.approx(math.dist(C1[c], C0[c]), rel=1e-15)
    assert np.array_equal(C1[k - 1], C0[k - 1]) and delta[k - 1] == 0.0


def test_beta_is_mean_block_box_diagonal():
    rng = np.random.default_rng(5)
    n, k = 3000, 8
    X = [rng.random(n), rng.random(n)]
    A = rng.integers(0, k - 2, n).astype(np.int32)  # two empty blocks
    diags = []
    for c in range(k - 2):
        m = A == c
        diags.append(math.hypot(X[0][m].max() - X[0][m].min(), X[1][m].max() - X[1][m].min()))
    assert oracle.beta(X, A, k) == pytest.approx(math.fsum(diags) / (k - 2), rel=1e-15)


def test_erosion_closed_forms():
    """alpha = 2/(1+exp(-delta/beta)) - 1 = tanh(delta / (2 beta)), and the
    influence becomes influence^(1 - alpha)."""
    beta = 0.25
    delta = np.array([0.0, beta, 1e3, 0.1, 0.1])
    I = np.array([1.7, 1.7, 0.4, 1.0, 0.6])
    out = oracle.erode(delta, beta, I)
    assert out[0] == 1.7                                     # no movement, no erosion
    assert out[1] == pytest.approx(1.7 ** (1 - math.tanh(0.5)), rel=1e-14)
    assert out[2] == pytest.approx(1.0, abs=1e-12)           # far move: back to 1
    assert out[3] == 1.0                                     # influence 1 is a fixed point
    assert out[4] == pytest.approx(0.6 ** (1 - math.tanh(0.2)), rel=1e-14)


def test_partition_stats():
    rng = np.random.default_rng(6)
    n, k = 4000, 5
    X = [rng.random(n), rng.random(n)]
    A = rng.integers(0, k - 1, n).astype(np.int32)
    st = oracle.partition_stats(X, A, k, 0.03)
    bw = np.bincount(A, minlength=k).astype(float)
    assert np.array_equal(st["block_weights"], bw)
    assert st["empty_blocks"] == 1
    assert st["imbalance"] == pytest.approx(bw.max() / (n / k) - 1)
    assert st["lmax"] == 1.03 * math.ceil(n / k)
    assert st["overloaded_blocks"] == int((bw > st["lmax"]).sum())
    obj = []
    for c in range(k - 1):
        m = A == c
        cx, cy = X[0][m].mean(), X[1][m].mean()
        obj.append(math.fsum((X[0][m] - cx) ** 2 + (X[1][m] - cy) ** 2))
    assert st["objective"] == pytest.approx(math.fsum(obj), rel=1e-12)
    assert np.all(np.isnan(st["centers"][k - 1]))
