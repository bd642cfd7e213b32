"""Pins of the graph-quality oracle (Sec. 2 block measures; Sec. 5.2
Metrics) on k-nearest-neighbour graphs: scipy's k-d tree, exact brute force
on lattices with ties, scipy's sparse symmetrisation, closed forms on grid
graphs, and networkx for cut, communication volume and diameters."""
import math

import numpy as np
import pytest

import oracle
from paper_1805_01208_amd import workloads


@pytest.mark.parametrize("d,K", [(2, 6), (3, 12), (2, 1)])
def test_knn_matches_scipy_kdtree(d, K):
    from scipy.spatial import cKDTree
    X = workloads.uniform(3000, d, 40 + d)
    nb = oracle.knn(X, K)
    P = np.stack(X, axis=1)
    _, idx = cKDTree(P).query(P, k=K + 1)
    # random points: no equal distances, so the point itself comes first
    assert np.array_equal(idx[:, 0], np.arange(3000))
    assert np.array_equal(nb, idx[:, 1:])


def test_knn_of_selected_points_is_their_rows():
    X = workloads.gauss3d(2000, 44)
    q = np.array([0, 17, 1999, 17, 640])
    assert np.array_equal(oracle.knn_of(X, 9, q), oracle.knn(X, 9)[q])


def test_knn_ties_on_a_lattice_by_exact_brute_force():
    """Integer lattice points: squared distances are exact integers, so
    sorting (distance, index) pairs in Python is the definition."""
    pts = [(x, y) for y in range(6) for x in range(7)]
    rng = np.random.default_rng(5)
    order = rng.permutation(len(pts))
    pts = [pts[i] for i in order]
    X = [np.array([p[0] for p in pts], float), np.array([p[1] for p in pts], float)]
    K = 8
    nb = oracle.knn(X, K)
    for i, (xi, yi) in enumerate(pts):
        ref = sorted(((xi - xj) ** 2 + (yi - yj) ** 2, j) for j, (xj, yj) in enumerate(pts) if j != i)
        assert list(nb[i]) == [j for _, j in ref[:K]]


def test_knn_duplicates_and_3d_lattice():
    pts = [(x, y, z) for z in range(3) for y in range(3) for x in range(3)] * 2
    X = [np.array([p[j] for p in pts], float) for j in range(3)]
    nb = oracle.knn(X, 7)
    for i, pi in enumerate(pts):
        ref = sorted((sum((a - b) ** 2 for a, b in zip(pi, pj)), j)
                     for j, pj in enumerate(pts) if j != i)
        assert list(nb[i]) == [j for _, j in ref[:7]]
    assert nb[0][0] == 27            # the duplicate of point 0 at distance 0


def test_symmetrize_matches_scipy_sparse():
    import scipy.sparse as sp
    X = workloads.gauss3d(2500, 41)
    nb = oracle.knn(X, 5)
    rp, col = oracle.knn_symmetrize(nb)
    n = nb.shape[0]
    M = sp.csr_matrix((np.ones(nb.size), (np.repeat(np.arange(n), 5), nb.ravel())), shape=(n, n))
    S = (M + M.T).tocsr()
    S.sort_indices()
    assert np.array_equal(rp, S.indptr) and np.array_equal(col, S.indices)
    assert np.all(np.diff(rp) >= 5)


def _grid_csr(a, b):
    """4-neighbour grid graph of a columns x b rows, vertex x + a*y."""
    rows = []
    for y in range(b):
        for x in range(a):
            nbrs = []
            if y > 0: nbrs.append(x + a * (y - 1))
            if x > 0: nbrs.append(x - 1 + a * y)
            if x < a - 1: nbrs.append(x + 1 + a * y)
            if y < b - 1: nbrs.append(x + a * (y + 1))
            rows.append(nbrs)
    rp = np.zeros(a * b + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    return rp, np.array([v for r in rows for v in r], dtype=np.int32)


def test_grid_strips_closed_forms():
    """a x b grid cut into s vertical strips of width w: cut (s-1)b, comm b
    for the two end strips and 2b inside, diameter (w-1)+(b-1)."""
    w, s, b = 5, 4, 7
    a = w * s
    rp, col = _grid_csr(a, b)
    A = np.array([(v % a) // w for v in range(a * b)], dtype=np.int32)
    m = oracle.graph_metrics(rp, col, A, s)
    assert m["edge_cut"] == (s - 1) * b
    assert list(m["comm"]) == [b] + [2 * b] * (s - 2) + [b]
    assert m["total_comm"] == 2 * (s - 1) * b and m["max_comm"] == 2 * b
    assert list(m["diameter"]) == [(w - 1) + (b - 1)] * s
    assert m["disconnected_blocks"] == 0
    assert m["harmonic_diameter"] == (w - 1) + (b - 1)


def test_disconnected_singleton_and_empty_blocks():
    """On the path 0-1-...-9: block 0 = {0, 4} (disconnected), block 1 =
    {1, 2, 3} (diameter 2), block 2 = {5..8} (diameter 3), block 3 = {9}
    (one vertex), block 4 empty.  Harmonic mean over blocks 0-2:
    3 / (0 + 1/2 + 1/3)."""
    rp, col = _grid_csr(10, 1)
    A = np.array([0, 1, 1, 1, 0, 2, 2, 2, 2, 3], dtype=np.int32)
    m = oracle.graph_metrics(rp, col, A, 5)
    assert list(m["diameter"]) == [-1, 2, 3, 0, 0]
    assert m["disconnected_blocks"] == 1 and m["max_diameter"] == 3
    assert m["harmonic_diameter"] == pytest.approx(3 / (1 / 2 + 1 / 3), rel=1e-15)
    # every block disconnected -> infinite harmonic mean; only singletons -> 0
    rp2, col2 = _grid_csr(4, 1)
    m2 = oracle.graph_metrics(rp2, col2, np.array([0, 1, 0, 1], np.int32), 2)
    assert m2["harmonic_diameter"] == math.inf
    m3 = oracle.graph_metrics(rp2, col2, np.array([0, 1, 2, 3], np.int32), 4)
    assert m3["harmonic_diameter"] == 0.0 and m3["edge_cut"] == 3


def test_metrics_match_networkx_on_a_knn_graph():
    import networkx as nx
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    X = workloads.uniform(1500, 2, 42)
    nb = oracle.knn(X, 6)
    rp, col = oracle.knn_symmetrize(nb)
    n, k = 1500, 9
    # a partition with ragged, partly disconnected blocks: vertical bands + a scatter
    A = np.minimum((X[0] * 8).astype(np.int32), 7)
    A[np.random.default_rng(43).random(n) < 0.01] = 8
    m = oracle.graph_metrics(rp, col, A, k)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    for u in range(n):
        for v in col[rp[u]:rp[u + 1]]:
            G.add_edge(u, int(v))
    blocks = [set(np.flatnonzero(A == b).tolist()) for b in range(k)]
    assert m["edge_cut"] == sum(nx.cut_size(G, blocks[b]) for b in range(k)) // 2
    for b in range(k):
        vol = sum(len({int(A[u]) for u in G[v]} - {b}) for v in blocks[b])
        assert m["comm"][b] == vol
        H = G.subgraph(blocks[b])
        if not nx.is_connected(H):
            assert m["diameter"][b] == -1
            continue
        exact = nx.diameter(H)
        assert exact >= m["diameter"][b] >= math.ceil(exact / 2)
        assert m["diameter_ub"][b] >= exact
        if m["diameter_ub"][b] == m["diameter"][b]:
            assert m["diameter"][b] == exact
        # never below the double sweep from the block's lowest vertex, with
        # scipy's breadth-first distances
        idx = sorted(blocks[b])
        pos = {v: i for i, v in enumerate(idx)}
        rows = [pos[u] for u in idx for v in G[u] if v in pos]
        cols = [pos[v] for u in idx for v in G[u] if v in pos]
        M = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(idx), len(idx)))
        d0 = shortest_path(M, unweighted=True, indices=0)
        far = int(np.flatnonzero(d0 == d0.max())[0])
        assert m["diameter"][b] >= int(shortest_path(M, unweighted=True, indices=far).max())


def _edges_csr(n, edges):
    rows = [[] for _ in range(n)]
    for u, v in edges:
        rows[u].append(v)
        rows[v].append(u)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    return rp, np.array([v for r in rows for v in sorted(r)], dtype=np.int32)


def _golden_traces():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ifub_traces.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[f[0]] = dict(zip(("a1", "b1", "r2", "a2", "b2", "u", "l", "rounds", "lb", "ub"),
                             map(int, f[1:])))
    return out


def test_diameter_bound_hand_traces():
    """4-sweep and iFUB rounds (Sec. 5.2, Metrics) traced by hand on three
    graphs: one where the double sweep from vertex 0 misses the diameter and
    one round closes the gap, a cycle that becomes exact in its third round,
    and a cycle still open after three rounds."""
    gold = _golden_traces()
    graphs = {
        "g7": _edges_csr(7, [(0, 4), (0, 6), (1, 4), (1, 6), (2, 6), (3, 6), (5, 6)]),
        "c12": _edges_csr(12, [(i, (i + 1) % 12) for i in range(12)]),
        "c14": _edges_csr(14, [(i, (i + 1) % 14) for i in range(14)]),
    }
    for name, (rp, col) in graphs.items():
        assert oracle.ifub_trace(rp, col) == gold[name], name
        m = oracle.graph_metrics(rp, col, np.zeros(len(rp) - 1, np.int32), 1)
        assert (m["diameter"][0], m["diameter_ub"][0]) == (gold[name]["lb"], gold[name]["ub"])
        assert m["exact_blocks"] == (1 if gold[name]["lb"] == gold[name]["ub"] else 0)


def test_diameter_bound_exact_on_paths_trees_grids_and_bounds_on_random_graphs():
    """Equal to the exact diameter (networkx) on paths, random trees and grids,
    where the first sweeps already reach it; on random connected graphs
    between the double sweep and the exact value, at most the proven upper
    bound, and exact whenever lower and upper bound meet."""
    import networkx as nx
    rng = np.random.default_rng(44)
    cases = [nx.path_graph(17), nx.grid_2d_graph(6, 9), nx.grid_2d_graph(1, 5)]
    cases += [nx.random_labeled_tree(int(rng.integers(2, 60)), seed=int(rng.integers(1 << 30)))
              for _ in range(20)]
    for G in cases:
        G = nx.convert_node_labels_to_integers(G, ordering="sorted")
        n = G.number_of_nodes()
        rp, col = _edges_csr(n, list(G.edges()))
        m = oracle.graph_metrics(rp, col, np.zeros(n, np.int32), 1)
        assert m["diameter"][0] == nx.diameter(G)
    seen_gap = 0
    for t in range(300):
        n = int(rng.integers(6, 40))
        G = nx.gnp_random_graph(n, float(rng.uniform(0.06, 0.3)), seed=int(rng.integers(1 << 30)))
        if not nx.is_connected(G):
            continue
        rp, col = _edges_csr(n, list(G.edges()))
        m = oracle.graph_metrics(rp, col, np.zeros(n, np.int32), 1)
        exact = nx.diameter(G)
        lb, ub = int(m["diameter"][0]), int(m["diameter_ub"][0])
        d0 = nx.single_source_shortest_path_length(G, 0)
        far = min(v for v in d0 if d0[v] == max(d0.values()))
        dsweep = max(nx.single_source_shortest_path_length(G, far).values())
        assert dsweep <= lb <= exact <= ub
        if lb == ub:
            assert lb == exact
        seen_gap += dsweep < exact
    assert seen_gap > 0


def test_invalid_graph_inputs():
    rp, col = _grid_csr(3, 3)
    with pytest.raises(RuntimeError):
        oracle.graph_metrics(rp, col, np.full(9, 2, np.int32), 2)
    bad = col.copy()
    bad[4] = 9
    with pytest.raises(RuntimeError):
        oracle.graph_metrics(rp, bad, np.zeros(9, np.int32), 1)
    with pytest.raises(RuntimeError):
        oracle.knn([np.zeros(4), np.zeros(4)], 4)
