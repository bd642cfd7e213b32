"""Pins of the oracle's Hilbert-curve bootstrap (Alg. 2, SFC index, sort and
initial centers) against the definition of the Hilbert curve, a hand-written
table of the classical curve, numpy's stable sort and a hand-worked index
example."""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hilbert_2d_order1_order2.txt")


def curve(d, m):
    """All cells of the order-m grid, in oracle key order; also the keys."""
    N = 1 << m
    cells = np.array(list(itertools.product(range(N), repeat=d)), dtype=np.uint32)
    keys = oracle.hilbert_indices(cells, m)
    order = np.argsort(keys, kind="stable")
    return cells[order], keys[order]


CASES = [(2, m) for m in range(1, 6)] + [(3, m) for m in range(1, 4)]


@pytest.mark.parametrize("d,m", CASES)
def test_bijection_onto_key_range(d, m):
    _, keys = curve(d, m)
    assert np.array_equal(keys, np.arange(1 << (d * m), dtype=np.uint64))


@pytest.mark.parametrize("d,m", CASES)
def test_consecutive_cells_are_face_neighbours(d, m):
    cells, _ = curve(d, m)
    steps = np.abs(np.diff(cells.astype(np.int64), axis=0)).sum(axis=1)
    assert np.all(steps == 1)


@pytest.mark.parametrize("d,m", CASES)
def test_aligned_key_runs_fill_aligned_subcubes(d, m):
    cells, _ = curve(d, m)
    for j in range(1, m + 1):
        run = 1 << (d * j)
        side = 1 << j
        for s in range(0, cells.shape[0], run):
            blk = cells[s:s + run].astype(np.int64)
            lo = blk.min(axis=0)
            assert np.all(lo % side == 0)
            assert np.all(blk.max(axis=0) - lo == side - 1)


@pytest.mark.parametrize("d,m", CASES)
def test_origin_has_key_zero(d, m):
    assert oracle.hilbert_index([0] * d, m) == 0


def _symmetries(d):
    """The 2^d * d! symmetries of the d-cube as (axis permutation, flips)."""
    for perm in itertools.permutations(range(d)):
        for flips in itertools.product((False, True), repeat=d):
            yield perm, flips


def _apply(cells, side, perm, flips):
    out = cells[:, list(perm)].copy()
    for a, f in enumerate(flips):
        if f:
            out[:, a] = side - 1 - out[:, a]
    return out


@pytest.mark.parametrize("d,m", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_recursive_definition(d, m):
    """The order-m curve is 2^d copies of the order-(m-1) curve, each turned
    by a symmetry of the cube and shifted into one sub-cube, visited in the
    order of the order-1 curve, each copy entering next to where the previous
    one left (the recursive construction of the Hilbert curve)."""
    big, _ = curve(d, m)
    small, _ = curve(d, m - 1)
    first, _ = curve(d, 1)
    half = 1 << (m - 1)
    n_sub = 1 << (d * (m - 1))
    for i in range(1 << d):
        part = big[i * n_sub:(i + 1) * n_sub].astype(np.int64)
        corner = part.min(axis=0)
        assert np.array_equal(corner // half, first[i].astype(np.int64))
        local = part - corner
        assert any(np.array_equal(_apply(small.astype(np.int64), half, p, f), local)
                   for p, f in _symmetries(d)), f"sub-cube {i} is not a turned copy"


def _golden():
    tables = {}
    cur = None
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("order"):
                cur = int(line.split()[1])
                continue
            tables[cur] = [tuple(int(v) for v in c.split(",")) for c in line.split()]
    return tables


@pytest.mark.parametrize("m", [1, 2])
def test_classical_curve_table(m):
    cells, _ = curve(2, m)
    assert [tuple(int(v) for v in c) for c in cells] == _golden()[m]


def test_keys_of_points_use_isotropic_cells():
    """Unit square at order 2: the cell of a point is floor(4*x) per axis
    (the largest extent sets the scale); the corner x=1 is clamped to cell 3."""
    X = [np.array([0.0, 1.0, 0.30, 0.99, 0.5]), np.array([0.0, 1.0, 0.80, 0.01, 0.5])]
    keys = oracle.sfc_keys(X, 2)
    table = {c: i for i, c in enumerate(_golden()[2])}
    expect = [table[(0, 0)], table[(3, 3)], table[(1, 3)], table[(3, 0)], table[(2, 2)]]
    assert list(keys) == expect


def test_anisotropic_box_scales_by_largest_extent():
    """A 4x1 box: both axes share the scale 2^m / 4, so y only reaches cell 0
    at order 2 (y < 1 -> floor(y) = 0)."""
    X = [np.array([0.0, 4.0, 2.0]), np.array([0.0, 1.0, 0.5])]
    keys = oracle.sfc_keys(X, 2)
    table = {c: i for i, c in enumerate(_golden()[2])}
    assert list(keys) == [table[(0, 0)], table[(3, 1)], table[(2, 0)]]


def test_zero_extent_gives_zero_keys():
    X = [np.full(7, 0.25), np.full(7, -3.0)]
    assert np.all(oracle.sfc_keys(X, 16) == 0)


def test_sort_is_numpy_stable_argsort():
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 50, 5000).astype(np.uint64)  # many equal keys
    assert np.array_equal(oracle.sfc_order(keys), np.argsort(keys, kind="stable"))


def test_initial_center_positions_worked_example():
    """n=10, k=3: sorted positions floor(i*10/3) + floor(10/6) = 1, 4, 7."""
    x = np.arange(10, dtype=np.float64)[::-1].copy()  # sorted order reverses the input
    X = [x, np.zeros(10)]
    centers, perm, keys = oracle.init_centers_sfc(X, 3, 8)
    assert np.array_equal(perm, np.argsort(keys, kind="stable"))
    assert list(centers[:, 0]) == [x[perm[1]], x[perm[4]], x[perm[7]]]
    assert list(centers[:, 0]) == [1.0, 4.0, 7.0]


@pytest.mark.parametrize("n,k", [(100, 1), (100, 100), (1000, 7), (12345, 64)])
def test_initial_centers_are_distinct_sorted_points(n, k):
    rng = np.random.default_rng(n + k)
    X = [rng.random(n), rng.random(n), rng.random(n)]
    centers, perm, keys = oracle.init_centers_sfc(X, k, 10)
    pos = np.array([(i * n) // k + n // (2 * k) for i in range(k)])
    assert len(set(pos)) == k and pos.max() < n
    for j in range(3):
        assert np.array_equal(centers[:, j], X[j][perm[pos]])
