"""End-to-end GPU balanced k-means (Alg. 2 around Alg. 1) against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import assert_assignment_parity, assert_centers_close, cuda, torch, widened
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def compare_run(X, k, eps, W=None, precision="f64", **kw):
    from paper_1805_01208_amd import bkm
    print(f"case d={len(X)} n={len(X[0])} k={k} eps={eps} weighted={W is not None} "
          f"{precision} {kw}", flush=True)
    Wt = None if W is None else torch.from_numpy(W).cuda()
    g = bkm.balanced_kmeans(cuda(X), k, W=Wt, eps=eps, precision=precision, **kw)
    okw = {kk: v for kk, v in kw.items() if kk in ("max_iter", "max_balance_iter", "erosion")}
    o = oracle.balanced_kmeans(widened(X), k, eps, W=W, **okw)
    A = g["A"].cpu().numpy()
    gi, oi = g["info"], o["info"]
    assert (gi["rounds"], gi["sweeps"], gi["balanced"], gi["converged"]) == (
        oi["rounds"], oi["sweeps"], oi["balanced"], oi["converged"])
    # the final assignment is the argmin under the state of the last sweep;
    # compare it with the oracle's and allow differences only at exact ties
    bad = np.flatnonzero(A != o["A"])
    assert bad.size == 0, f"{bad.size} assignments differ"
    assert_centers_close(g["centers"].cpu().numpy(), o["centers"], X, "centers")
    assert np.allclose(g["influence"].cpu().numpy(), o["influence"], rtol=1e-12, atol=0)
    if W is None:
        assert np.array_equal(g["block_weights"].cpu().numpy(), o["block_weights"])
    else:
        assert np.allclose(g["block_weights"].cpu().numpy(), o["block_weights"], rtol=1e-13)
    return g, o


@pytest.mark.parametrize("precision", ["f64", "f32_recheck"])
def test_c1_uniform_2d(precision):
    cfg = workloads.c1()
    g, o = compare_run(cfg["X"], cfg["k"], cfg["eps"], precision=precision)
    assert g["info"]["balanced"] == 1
    assert g["info"]["skipped"] > 0


@pytest.mark.parametrize("precision", ["f64", "f32_recheck"])
def test_refined_2d_k64(precision):
    X = workloads.refined2d(120000, 2)
    compare_run(X, 64, 0.03, precision=precision, max_iter=20)


@pytest.mark.parametrize("precision", ["f64", "f32_recheck"])
def test_erosion_off(precision):
    """Without erosion the influence is kept from round to round."""
    X = workloads.gauss3d(20000, 37)
    g, o = compare_run(X, 24, 0.02, precision=precision, max_iter=20, erosion=False)
    e = oracle.balanced_kmeans(widened(X), 24, 0.02, max_iter=20)
    assert not np.array_equal(o["influence"], e["influence"])


def test_weighted_3d():
    rng = np.random.default_rng(8)
    X = workloads.gauss3d(50000, 8)
    W = rng.lognormal(0.0, 0.5, 50000)
    compare_run(X, 24, 0.05, W=W, precision="f32_recheck", max_iter=20)


def test_single_block():
    rng = np.random.default_rng(3)
    X = [rng.random(3000), rng.random(3000), rng.random(3000)]
    g, o = compare_run(X, 1, 0.03)
    assert np.all(g["A"].cpu().numpy() == 0)


def test_every_point_its_own_block():
    rng = np.random.default_rng(4)
    X = [rng.random(700), rng.random(700)]
    compare_run(X, 700, 0.03, max_iter=3)


def test_float32_input_matches_widened_oracle():
    rng = np.random.default_rng(5)
    X = [rng.random(40000).astype(np.float32) for _ in range(2)]
    compare_run(X, 16, 0.03, precision="f32_recheck", max_iter=15)


def test_partition_stats_matches_oracle():
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(6)
    n, k = 50000, 37
    X = [rng.random(n) for _ in range(3)]
    W = rng.lognormal(0, 0.5, n)
    A = rng.integers(0, k - 1, n).astype(np.int32)  # block k-1 empty
    for w in (None, W):
        st = bkm.partition_stats(cuda(X), torch.from_numpy(A).cuda(), k, 0.03,
                                 W=None if w is None else torch.from_numpy(w).cuda())
        o = oracle.partition_stats(X, A, k, 0.03, W=w)
        assert st["empty_blocks"] == o["empty_blocks"] == 1
        assert st["overloaded_blocks"] == o["overloaded_blocks"]
        assert st["imbalance"] == pytest.approx(o["imbalance"], rel=1e-12)
        assert st["objective"] == pytest.approx(o["objective"], rel=1e-12)
        if w is None:
            assert st["l_max"] == o["lmax"]
        else:  # total node weight: GPU tree sum vs compensated sum, within an ulp or two
            assert st["l_max"] == pytest.approx(o["lmax"], rel=4e-16)
        bw = st["block_weights"].cpu().numpy()
        assert np.allclose(bw, o["block_weights"], rtol=1e-13, atol=0)
        c = st["centers"].cpu().numpy()
        assert np.all(np.isnan(c[k - 1]))
        assert_centers_close(c[:k - 1], o["centers"][:k - 1], X, "stats centers")
    bad = A.copy()
    bad[5] = k
    with pytest.raises(bkm.BkmError):
        bkm.partition_stats(cuda(X), torch.from_numpy(bad).cuda(), k)


@pytest.mark.parametrize("precision", ["f64", "f32_recheck"])
def test_kept_candidate_lists(precision):
    """Balance sweeps keep the candidate lists of a round's first sweep while
    the influences move within the lists' margin (Sec. 4.4 filter, widened):
    a run that keeps them in some sweeps and rebuilds them in others equals
    the oracle's run."""
    X = workloads.shells3d(400000, 5)
    g, _ = compare_run(X, 96, 0.01, precision=precision, max_iter=15)
    gi = g["info"]
    print(f"  sweeps {gi['sweeps']}, list builds {gi['list_builds']}", flush=True)
    assert gi["rounds"] <= gi["list_builds"] < gi["sweeps"]
