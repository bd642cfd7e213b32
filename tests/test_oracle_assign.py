"""Pins of the oracle's assignment (argmin of the effective distance
dist(p, c) / influence(c), Sec. 4.2) against a k-d tree nearest-neighbour
query, the Apollonius-circle closed form of the two-center weighted Voronoi
diagram, a brute force built on math.dist, and invariances."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle


def cloud(n, d, seed):
    rng = np.random.default_rng(seed)
    return [rng.random(n) for _ in range(d)]


@pytest.mark.parametrize("d", [2, 3])
def test_unit_influence_is_nearest_neighbour(d):
    X = cloud(20000, d, 1 + d)
    C = np.stack(cloud(300, d, 7 + d), axis=1)
    A, best, second = oracle.assign(X, C, np.ones(300))
    dist, idx = cKDTree(C).query(np.stack(X, axis=1), k=2)
    assert np.array_equal(A, idx[:, 0])
    assert np.allclose(best, dist[:, 0], rtol=1e-14, atol=0)
    assert np.allclose(second, dist[:, 1], rtol=1e-14, atol=0)


@pytest.mark.parametrize("d", [2, 3])
def test_two_centers_apollonius_sphere(d):
    """With influences I0 < I1 the points of center 0 are exactly those inside
    the Apollonius sphere |p-c0| / |p-c1| = rho = I0/I1, whose center is
    (c0 - rho^2 c1) / (1 - rho^2) and radius rho |c0-c1| / (1 - rho^2)."""
    rng = np.random.default_rng(5)
    c0 = rng.random(d)
    c1 = rng.random(d)
    I = np.array([0.7, 1.3])
    rho = I[0] / I[1]
    mid = (c0 - rho ** 2 * c1) / (1 - rho ** 2)
    rad = rho * np.linalg.norm(c0 - c1) / (1 - rho ** 2)
    P = rng.uniform(-2, 3, (30000, d))
    r = np.linalg.norm(P - mid, axis=1)
    far = np.abs(r - rad) > 1e-9 * rad  # drop points numerically on the sphere
    X = [P[far, j].copy() for j in range(d)]
    A, _, _ = oracle.assign(X, np.stack([c0, c1]), I)
    assert np.array_equal(A == 0, r[far] < rad)
    assert 0 < (A == 0).sum() < far.sum()


def test_brute_force_with_math_dist():
    rng = np.random.default_rng(3)
    for d in (2, 3):
        X = [rng.random(60) for _ in range(d)]
        C = rng.random((9, d))
        I = rng.uniform(0.5, 2.0, 9)
        A, best, second = oracle.assign(X, C, I)
        for i in range(60):
            p = [X[j][i] for j in range(d)]
            eff = sorted((math.dist(p, C[c]) / I[c], c) for c in range(9))
            assert A[i] == eff[0][1]
            assert best[i] == pytest.approx(eff[0][0], rel=1e-15)
            assert second[i] == pytest.approx(eff[1][0], rel=1e-15)


def test_uniform_influence_scale_does_not_change_assignment():
    X = cloud(10000, 3, 9)
    C = np.stack(cloud(50, 3, 10), axis=1)
    I = np.random.default_rng(2).uniform(0.8, 1.2, 50)
    A1, _, _ = oracle.assign(X, C, I)
    A2, _, _ = oracle.assign(X, C, I * 4.0)  # power of two: exact rescale
    assert np.array_equal(A1, A2)


def test_larger_influence_grows_its_cell():
    X = cloud(20000, 2, 4)
    C = np.stack(cloud(20, 2, 5), axis=1)
    I = np.ones(20)
    A1, _, _ = oracle.assign(X, C, I)
    I[3] = 1.2
    A2, _, _ = oracle.assign(X, C, I)
    assert (A2 == 3).sum() > (A1 == 3).sum()
    assert np.all(A2[A1 == 3] == 3)  # nobody leaves the grown cell


def test_ties_go_to_lowest_index():
    X = cloud(500, 2, 6)
    c = np.array([0.5, 0.5])
    C = np.stack([c, c, np.array([5.0, 5.0])])
    A, best, second = oracle.assign(X, C, np.ones(3))
    assert np.all(A == 0)
    assert np.array_equal(best, second)


def test_single_center():
    X = cloud(100, 3, 8)
    A, best, second = oracle.assign(X, np.array([[0.1, 0.2, 0.3]]), np.array([2.0]))
    assert np.all(A == 0)
    assert np.all(np.isinf(second))
    assert np.allclose(best, np.linalg.norm(np.stack(X, 1) - [0.1, 0.2, 0.3], axis=1) / 2.0)


def test_third_dimension_counts():
    """Two centers that differ only in z: a dropped z term would tie them."""
    X = [np.array([0.5]), np.array([0.5]), np.array([0.9])]
    C = np.array([[0.5, 0.5, 0.0], [0.5, 0.5, 1.0]])
    A, best, _ = oracle.assign(X, C, np.ones(2))
    assert A[0] == 1 and best[0] == pytest.approx(0.1, rel=1e-12)
