"""Parity at the full sizes of the benchmark workloads, in the launch
configuration the benchmark times (default tile size; FP32 screen + FP64
recheck, and plain FP64 on the 2D refined cloud).

The oracle cannot run these sizes end to end (a brute-force sweep of the 3D
shell cloud is 2.6e11 distance evaluations), so the checks are:
  * Hilbert keys of every point against the oracle's keys (bit-exact), the
    sort order and the initial centers against their definitions (Alg. 2);
  * sweeps with injected states (Alg. 1, bounds carried across steps):
    assignments against the oracle's brute-force argmin (Sec. 4.2) -- of
    every point of the 2D refined cloud (16M, both precisions), of an 8M
    random sample of the 3D shell cloud and a 1M sample of the 250M cloud
    (the oracle takes about 2e9 point-center pairs per second on 16 host
    threads; all 64M x 4096 pairs would take over two minutes per step) --
    block weights of every step against an exact count;
  * the batched workload's full recipe (256 instances of up to 2M points):
    every instance identical to its separate run, the smallest ones also to
    the oracle's run;
  * full runs: block weights against an exact recount, centers against the
    weighted means of their blocks (Alg. 2), the balance bound when balanced.
"""
import numpy as np
import pytest

import oracle
from gpu_common import assert_assignment_parity, cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]

SAMPLE_C3 = 8_000_000
SAMPLE_C5 = 1_000_000


@pytest.fixture(scope="module")
def c2():
    cfg = workloads.c2()
    return cfg, cuda(cfg["X"])


@pytest.fixture(scope="module")
def c3():
    cfg = workloads.c3()
    return cfg, cuda(cfg["X"])


@pytest.fixture(scope="module")
def c5():
    cfg = workloads.c5()
    return cfg, cuda(cfg["X"]), torch.from_numpy(cfg["W"]).cuda()


def check_bootstrap(cfg, X):
    from paper_1805_01208_amd import bkm
    k = cfg["k"]
    print(f"case full-size bootstrap {cfg['name']} k={k}", flush=True)
    Xw = widened(cfg["X"])
    n = len(Xw[0])
    cen, perm, keys = bkm.init_centers_sfc(X, k, 16)
    keys = keys.cpu().numpy().view(np.uint64)
    perm = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(keys, oracle.sfc_keys(Xw, 16))
    # a permutation, sorted by (key, input index)
    assert np.all(np.bincount(perm, minlength=n) == 1)
    ks = keys[perm]
    assert np.all(ks[1:] >= ks[:-1])
    tie = ks[1:] == ks[:-1]
    assert np.all(perm[1:][tie] > perm[:-1][tie])
    pos = (np.arange(k, dtype=np.int64) * n) // k + n // (2 * k)
    ref = np.stack([x[perm[pos]] for x in Xw], axis=1)
    assert np.array_equal(cen.cpu().numpy(), ref)
    return ref


def check_sweeps(cfg, X, C0, precision, seed, sample=None):
    from paper_1805_01208_amd import bkm
    k = cfg["k"]
    Xw = widened(cfg["X"])
    n = len(Xw[0])
    ext = max(float(x.max() - x.min()) for x in Xw)
    rng = np.random.default_rng(seed)
    Cs = [C0, C0 + rng.normal(0.0, 0.002 * ext, C0.shape),
          C0 + rng.normal(0.0, 0.01 * ext, C0.shape)]
    Is = [np.ones(k), rng.uniform(0.95, 1.05, k), rng.uniform(0.8, 1.25, k)]
    print(f"case full-size sweeps {cfg['name']} n={n} k={k} {precision}", flush=True)
    A, bw, info = bkm.assign_sweeps(X, torch.from_numpy(np.stack(Cs)), torch.from_numpy(np.stack(Is)),
                                    precision=precision)
    A = A.cpu().numpy()
    bw = bw.cpu().numpy()
    idx = np.arange(n) if sample is None else np.sort(rng.choice(n, size=sample, replace=False))
    Xs = Xw if sample is None else [x[idx] for x in Xw]
    for s in range(len(Cs)):
        print(f"  step {s}: oracle on {len(idx)} points", flush=True)
        Ao, best, second = oracle.assign(Xs, Cs[s], Is[s])
        assert_assignment_parity(A[s][idx], Ao, best, second, f"step {s}", Xs, Cs[s], Is[s])
        assert np.array_equal(bw[s], np.bincount(A[s], minlength=k).astype(np.float64))
    assert info["skipped"] > 0
    return info


def check_run(cfg, X, W=None, precision="f32_recheck"):
    from paper_1805_01208_amd import bkm
    k = cfg["k"]
    Xw = widened(cfg["X"])
    Wh = cfg["W"]
    print(f"case full-size run {cfg['name']} k={k} {precision}", flush=True)
    g = bkm.balanced_kmeans(X, k, W=W, eps=cfg["eps"], max_iter=50, precision=precision)
    A = g["A"].cpu().numpy()
    assert A.min() >= 0 and A.max() < k
    if Wh is None:
        cnt = np.bincount(A, minlength=k).astype(np.float64)
        assert np.array_equal(g["block_weights"].cpu().numpy(), cnt)
        wsum = cnt
    else:
        wsum = np.bincount(A, weights=Wh, minlength=k)
        assert np.allclose(g["block_weights"].cpu().numpy(), wsum, rtol=1e-12, atol=0)
    C = g["centers"].cpu().numpy()
    ext = max(float(x.max() - x.min()) for x in Xw)
    for j, x in enumerate(Xw):
        s = np.bincount(A, weights=x if Wh is None else Wh * x, minlength=k)
        ref = s / np.where(wsum > 0, wsum, 1.0)
        ne = wsum > 0
        err = np.max(np.abs(C[ne, j] - ref[ne]))
        assert err <= 1e-10 * max(ext, float(np.max(np.abs(ref[ne])))), f"axis {j}: {err}"
    if g["info"]["balanced"]:
        assert wsum.max() <= g["info"]["l_max"]
    return g


def test_c2_refined2d_16M(c2):
    cfg, X = c2
    C0 = check_bootstrap(cfg, X)
    for prec, seed in (("f64", 21), ("f32_recheck", 22)):
        check_sweeps(cfg, X, C0, prec, seed)
    g = check_run(cfg, X, precision="f64")
    assert g["info"]["balanced"] == 1


def test_c3_shells3d_64M(c3):
    cfg, X = c3
    C0 = check_bootstrap(cfg, X)
    check_sweeps(cfg, X, C0, "f32_recheck", 31, SAMPLE_C3)
    g = check_run(cfg, X)
    assert g["info"]["balanced"] == 1


def test_c5_radial2d_250M_weighted(c5):
    cfg, X, W = c5
    C0 = check_bootstrap(cfg, X)
    check_sweeps(cfg, X, C0, "f32_recheck", 51, SAMPLE_C5)
    check_run(cfg, X, W=W)


def check_knn_graph(cfg, X, K, A=None, k=None):
    """Exact K-NN lists of sampled points against the oracle's brute force
    over the whole cloud; the CSR graph against its definition on the
    sampled rows; the metrics of a partition against the oracle's metrics
    of the same CSR graph."""
    from paper_1805_01208_amd import bkm
    Xw = widened(cfg["X"])
    n = len(Xw[0])
    print(f"case full-size knn graph {cfg['name']} K={K}", flush=True)
    nbr, info = bkm.knn(X, K, order=True)
    order = info["order"]
    assert torch.equal(torch.sort(order.long()).values, torch.arange(n, device=order.device))
    rng = np.random.default_rng(91)
    q = np.sort(rng.choice(n, size=300, replace=False))
    nb = nbr.cpu().numpy()
    assert np.array_equal(nb[q], oracle.knn_of(Xw, K, q))
    rp, col = bkm.knn_graph(nbr, order)
    rph, colh = rp.cpu().numpy(), col.cpu().numpy()
    assert rph[0] == 0 and rph[-1] == len(colh) and np.all(np.diff(rph) >= K)
    for u in q[:50]:
        row = colh[rph[u]:rph[u + 1]]
        assert np.all(row[1:] > row[:-1])                     # sorted, no duplicates
        assert set(nb[u]) <= set(row.tolist())
        for v in row:                                          # every entry is a kNN relation
            assert v in nb[u] or u in nb[v]
    if A is not None:
        print(f"case full-size graph metrics {cfg['name']} k={k}", flush=True)
        g = bkm.graph_metrics(rp, col, A, k)
        o = oracle.graph_metrics(rph, colh, A.cpu().numpy(), k)
        for key in ("edge_cut", "max_comm", "total_comm", "max_diameter", "disconnected_blocks",
                    "exact_blocks"):
            assert g[key] == o[key], key
        assert np.array_equal(g["diameter"].cpu().numpy(), o["diameter"])
        assert np.array_equal(g["diameter_ub"].cpu().numpy(), o["diameter_ub"])
    return info


def test_c2_knn_graph_and_metrics(c2):
    from paper_1805_01208_amd import bkm
    cfg, X = c2
    part = bkm.balanced_kmeans(X, cfg["k"], eps=cfg["eps"], max_iter=20)
    check_knn_graph(cfg, X, 6, part["A"], cfg["k"])


def test_c3_knn(c3):
    cfg, X = c3
    check_knn_graph(cfg, X, 10)


def test_c4_batched_full_recipe():
    """The batched workload as the benchmark defines it: 256 instances, n
    log-uniform in [1e4, 2e6], k log-uniform in [8, 512], even ids 2D
    uniform, odd ids 3D Gaussian clusters, FP32+recheck, tiles from the
    autotuner.  Every instance must equal its separate run; the four
    smallest also the oracle's run."""
    from paper_1805_01208_amd import bkm
    cfgs = workloads.c4()
    insts = [(cuda(c["X"]), c["k"]) for c in cfgs]
    print(f"case full-size batched C4: {len(insts)} instances, "
          f"{sum(len(c['X'][0]) for c in cfgs)} points", flush=True)
    outs, rc = bkm.balanced_kmeans_batched(insts, max_iter=50)
    assert rc in (0, 1)
    for i, (inst, res) in enumerate(zip(insts, outs)):
        g = bkm.balanced_kmeans(inst[0], inst[1], max_iter=50)
        assert torch.equal(res["A"], g["A"]), f"instance {i}"
        assert torch.equal(res["centers"], g["centers"]), f"instance {i}"
        assert (res["info"]["rounds"], res["info"]["sweeps"]) == (g["info"]["rounds"],
                                                                  g["info"]["sweeps"])
    small = sorted(range(len(cfgs)), key=lambda i: len(cfgs[i]["X"][0]))[:4]
    for i in small:
        c = cfgs[i]
        print(f"  oracle instance {i}: n={len(c['X'][0])} k={c['k']}", flush=True)
        o = oracle.balanced_kmeans(widened(c["X"]), c["k"], 0.03, max_iter=50)
        assert np.array_equal(outs[i]["A"].cpu().numpy(), o["A"]), f"instance {i}"
        assert (outs[i]["info"]["rounds"], outs[i]["info"]["sweeps"]) == (o["info"]["rounds"],
                                                                          o["info"]["sweeps"])
