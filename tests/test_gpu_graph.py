"""Graph-quality evaluation on the GPU (Sec. 2 block measures; Sec. 5.2
Metrics): exact k-nearest-neighbour lists, their undirected CSR graph, and
edge cut / communication volume / block diameter bounds, each identical to
the oracle's."""
import numpy as np
import pytest

import oracle
from gpu_common import cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def _knn_both(X, K, what):
    from paper_1805_01208_amd import bkm
    print(f"case graph knn {what} n={len(X[0])} d={len(X)} K={K}", flush=True)
    nbr, info = bkm.knn(cuda(X), K)
    ref = oracle.knn(widened(X), K)
    assert np.array_equal(nbr.cpu().numpy(), ref), what
    assert info["group_visits"] > 0 and info["search_ms"] > 0
    return nbr, ref


@pytest.mark.parametrize("d,K,seed", [(2, 6, 1), (3, 12, 2), (2, 16, 3), (3, 1, 4)])
def test_knn_uniform(d, K, seed):
    _knn_both(workloads.uniform(20000, d, 60 + seed), K, "uniform")


def test_knn_clustered_and_f32():
    _knn_both(workloads.refined2d(30000, 65), 8, "refined2d")
    _knn_both([x.astype(np.float32) for x in workloads.gauss3d(15000, 66)], 10, "gauss3d f32")


def test_knn_lattice_ties_and_duplicates():
    """Many equal distances (integer lattice, shuffled) and duplicate points:
    ties go to the lower input index on both sides."""
    rng = np.random.default_rng(67)
    gx, gy = np.meshgrid(np.arange(150.0), np.arange(120.0))
    P = np.stack([gx.ravel(), gy.ravel()], axis=1)
    P = np.concatenate([P, P[rng.choice(len(P), 500, replace=False)]])
    P = P[rng.permutation(len(P))]
    _knn_both([P[:, 0].copy(), P[:, 1].copy()], 8, "lattice")
    g3 = np.stack(np.meshgrid(np.arange(20.0), np.arange(20.0), np.arange(12.0)), -1).reshape(-1, 3)
    g3 = g3[rng.permutation(len(g3))]
    _knn_both([g3[:, j].copy() for j in range(3)], 14, "lattice3d")


def test_knn_extreme_scales_and_near_ties():
    """The search screens partners with a fused squared distance against a
    slightly widened limit and decides with the exact one: clouds whose
    squared distances are subnormal or near 1e300, and pairs of points one
    unit in the last place apart, must still give the oracle's lists."""
    rng = np.random.default_rng(71)
    base = workloads.uniform(6000, 3, 72)
    _knn_both([x * 1e-160 for x in base], 7, "scale 1e-160")
    _knn_both([x * 1e150 for x in base], 7, "scale 1e150")
    P = np.stack(workloads.uniform(3000, 2, 73), axis=1)
    Q = np.nextafter(P, np.inf)
    R = P + rng.choice([-1.0, 1.0], P.shape) * np.spacing(P) * rng.integers(0, 3, P.shape)
    M = np.concatenate([P, Q, R])[rng.permutation(3 * len(P))]
    _knn_both([M[:, 0].copy(), M[:, 1].copy()], 5, "ulp neighbours")


@pytest.mark.parametrize("n,K", [(2, 1), (5, 4), (17, 16), (65, 1), (300, 16), (1025, 7)])
def test_knn_small_and_ragged(n, K):
    _knn_both(workloads.uniform(n, 2, 68 + n), K, "small")


def test_knn_graph_matches_oracle():
    from paper_1805_01208_amd import bkm
    X = workloads.gauss3d(12000, 69)
    nbr, ref = _knn_both(X, 9, "for graph")
    orp, ocol = oracle.knn_symmetrize(ref)
    nb2, info = bkm.knn(cuda(X), 9, order=True)
    assert torch.equal(nb2, nbr)
    order = info["order"]
    assert np.array_equal(np.sort(order.cpu().numpy()), np.arange(len(X[0])))
    rng = np.random.default_rng(74)
    shuffled = torch.from_numpy(rng.permutation(len(X[0])).astype(np.int32)).cuda()
    for o in (None, order, shuffled):
        rp, col = bkm.knn_graph(nbr, o)
        assert np.array_equal(rp.cpu().numpy(), orp)
        assert np.array_equal(col.cpu().numpy(), ocol)


def _metrics_both(rp, col, A, k, what):
    from paper_1805_01208_amd import bkm
    print(f"case graph metrics {what} k={k}", flush=True)
    g = bkm.graph_metrics(rp, col, A, k)
    o = oracle.graph_metrics(rp.cpu().numpy(), col.cpu().numpy(), A.cpu().numpy(), k)
    for key in ("edge_cut", "max_comm", "total_comm", "max_diameter", "disconnected_blocks",
                "exact_blocks"):
        assert g[key] == o[key], (what, key)
    assert np.array_equal(g["comm"].cpu().numpy(), o["comm"])
    assert np.array_equal(g["diameter"].cpu().numpy(), o["diameter"])
    assert np.array_equal(g["diameter_ub"].cpu().numpy(), o["diameter_ub"])
    if np.isfinite(o["harmonic_diameter"]):
        assert g["harmonic_diameter"] == pytest.approx(o["harmonic_diameter"], rel=1e-12)
    else:
        assert g["harmonic_diameter"] == o["harmonic_diameter"]
    return g


def test_metrics_of_partitions_match_oracle():
    from paper_1805_01208_amd import bkm
    X = workloads.uniform(25000, 2, 70)
    Xd = cuda(X)
    nbr, _ = bkm.knn(Xd, 6)
    rp, col = bkm.knn_graph(nbr)
    part = bkm.balanced_kmeans(Xd, 32, max_iter=20)
    g = _metrics_both(rp, col, part["A"], 32, "balanced k-means")
    assert g["bfs_levels"] > 0
    rng = np.random.default_rng(71)
    A = torch.from_numpy(rng.integers(0, 7, 25000).astype(np.int32)).cuda()
    _metrics_both(rp, col, A, 7, "random blocks")
    A = torch.from_numpy((X[0] * 5).astype(np.int32)).cuda()
    _metrics_both(rp, col, A, 9, "bands, empty blocks 5-8")
    _metrics_both(rp, col, torch.zeros(25000, dtype=torch.int32).cuda(), 1, "one block")


def test_metrics_with_more_connected_blocks_than_cus():
    """More connected blocks than compute units: the second launch of the
    diameter searches then takes them in the order of their first search's
    length.  Results identical to the oracle's."""
    from paper_1805_01208_amd import bkm
    X = workloads.uniform(96000, 2, 76)
    Xd = cuda(X)
    nbr, info = bkm.knn(Xd, 6, order=True)
    rp, col = bkm.knn_graph(nbr, info["order"])
    part = bkm.balanced_kmeans(Xd, 480, max_iter=20)
    g = _metrics_both(rp, col, part["A"], 480, "480 blocks")
    assert 480 - g["disconnected_blocks"] > torch.cuda.get_device_properties(0).multi_processor_count


def test_metrics_on_a_grid_graph():
    """The 4-neighbour grid in strips: closed forms on both sides."""
    w, s, b = 6, 5, 9
    a = w * s
    rows = []
    for y in range(b):
        for x in range(a):
            rows.append([v for v, ok in ((x + a * (y - 1), y > 0), (x - 1 + a * y, x > 0),
                                         (x + 1 + a * y, x < a - 1), (x + a * (y + 1), y < b - 1)) if ok])
    rp = torch.tensor(np.concatenate([[0], np.cumsum([len(r) for r in rows])]), dtype=torch.int64).cuda()
    col = torch.tensor([v for r in rows for v in r], dtype=torch.int32).cuda()
    A = torch.tensor([(v % a) // w for v in range(a * b)], dtype=torch.int32).cuda()
    g = _metrics_both(rp, col, A, s, "grid strips")
    assert g["edge_cut"] == (s - 1) * b and g["max_diameter"] == (w - 1) + (b - 1)


def _csr_of_edges(n, edges):
    rows = [[] for _ in range(n)]
    for u, v in edges:
        rows[u].append(v)
        rows[v].append(u)
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    col = np.array([v for r in rows for v in sorted(r)], dtype=np.int32)
    return torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()


def test_diameter_rounds_with_large_fringes():
    """Blocks that stay open through all three iFUB rounds, with fringes of
    up to 199 vertices (several 64-source passes): products of a cycle and
    a complete graph (every vertex has the same eccentricity), a long cycle
    (still open after three rounds), a path, and random sparse blocks; the
    bounds, upper bounds and exact counts must equal the oracle's."""
    import networkx as nx
    rng = np.random.default_rng(73)
    parts = [nx.cartesian_product(nx.cycle_graph(10), nx.complete_graph(100)),
             nx.cartesian_product(nx.cycle_graph(14), nx.complete_graph(80)),
             nx.cycle_graph(40), nx.path_graph(33)]
    parts += [nx.gnp_random_graph(int(rng.integers(20, 200)), 0.05, seed=int(rng.integers(1 << 30)))
              for _ in range(12)]
    edges, A, base = [], [], 0
    for b, G in enumerate(parts):
        G = nx.convert_node_labels_to_integers(G, ordering="sorted")
        edges += [(u + base, v + base) for u, v in G.edges()]
        A += [b] * G.number_of_nodes()
        base += G.number_of_nodes()
    # shuffle vertex ids so that blocks interleave in the index order
    perm = rng.permutation(base)
    edges = [(int(perm[u]), int(perm[v])) for u, v in edges]
    Ap = np.empty(base, dtype=np.int32)
    Ap[perm] = np.array(A, dtype=np.int32)
    # a few edges between blocks (they only add to the cut)
    for _ in range(30):
        u, v = rng.integers(0, base, 2)
        if Ap[u] != Ap[v]:
            edges.append((int(u), int(v)))
    rp, col = _csr_of_edges(base, edges)
    g = _metrics_both(rp, col, torch.from_numpy(Ap).cuda(), len(parts), "large fringes")
    d = g["diameter"].cpu().numpy()
    dub = g["diameter_ub"].cpu().numpy()
    assert (d[0], dub[0]) == (6, 6) and (d[1], dub[1]) == (8, 10)
    assert (d[2], dub[2]) == (20, 34)


def test_invalid_graph_inputs_are_rejected():
    from paper_1805_01208_amd import bkm
    X = cuda(workloads.uniform(3000, 2, 72))
    nbr, _ = bkm.knn(X, 4)
    rp, col = bkm.knn_graph(nbr)
    with pytest.raises(bkm.BkmError, match="assignment"):
        bkm.graph_metrics(rp, col, torch.full((3000,), 3, dtype=torch.int32).cuda(), 3)
    bad = col.clone()
    bad[10] = 3000
    with pytest.raises(bkm.BkmError, match="row_ptr/col"):
        bkm.graph_metrics(rp, bad, torch.zeros(3000, dtype=torch.int32).cuda(), 1)
    nb2 = nbr.clone()
    nb2[7, 2] = 7
    with pytest.raises(bkm.BkmError, match="neighbour"):
        bkm.knn_graph(nb2)
    nb2[7, 2] = -1
    with pytest.raises(bkm.BkmError, match="neighbour"):
        bkm.knn_graph(nb2)
    # vertex orders that are not permutations of 0..n-1
    dup = torch.arange(3000, dtype=torch.int32).cuda()
    dup[5] = 6
    out = torch.arange(3000, dtype=torch.int32).cuda()
    out[9] = 3000
    for o in (dup, out):
        with pytest.raises(bkm.BkmError, match="permutation"):
            bkm.knn_graph(nbr, o)
    # and the check leaves nothing behind: a valid order right after works
    rp2, col2 = bkm.knn_graph(nbr, torch.arange(3000, dtype=torch.int32).cuda())
    assert torch.equal(rp2, rp) and torch.equal(col2, col)
