"""The no-allocation statistics entry point against bkm_partition_stats, called
through the C ABI: two calls in a row, the second on a smaller input, and
the workspace limit."""
import numpy as np
import pytest

from gpu_common import cuda, torch
from paper_1805_01208_amd import workloads

pytestmark = pytest.mark.gpu


def compare(X, A, k, W=None, target_sizes=None, eps=0.03):
    from paper_1805_01208_amd import bkm
    print(f"case noalloc stats n={len(X[0])} k={k} weighted={W is not None} "
          f"targets={target_sizes is not None}", flush=True)
    Xg = cuda(X)
    Wg = None if W is None else torch.from_numpy(W).cuda()
    Ag = torch.from_numpy(A).cuda()
    ref = bkm.partition_stats(Xg, Ag, k, eps=eps, W=Wg, target_sizes=target_sizes)
    # outputs preallocated by the caller: the call itself allocates nothing
    bw = torch.full((k,), -1.0, dtype=torch.float64, device="cuda")
    cen = torch.full((k, len(X)), -1.0, dtype=torch.float64, device="cuda")
    got = bkm.partition_stats_noalloc(Xg, Ag, k, eps=eps, W=Wg, target_sizes=target_sizes,
                                      bw=bw, cen=cen)
    for key in ("imbalance", "objective", "l_max", "empty_blocks", "overloaded_blocks"):
        assert got[key] == ref[key], key
    assert np.array_equal(got["block_weights"].cpu().numpy(), ref["block_weights"].cpu().numpy())
    assert np.array_equal(got["centers"].cpu().numpy(), ref["centers"].cpu().numpy(),
                          equal_nan=True)
    if W is None:
        cnt = np.bincount(A, minlength=k).astype(np.float64)
        assert np.array_equal(got["block_weights"].cpu().numpy(), cnt)
    return got


def test_noalloc_stats_two_calls_second_smaller():
    rng = np.random.default_rng(3)
    X = workloads.gauss3d(200000, 4)
    k = 700
    A = rng.integers(0, k, len(X[0])).astype(np.int32)
    W = rng.lognormal(0.0, 0.5, len(X[0]))
    compare(X, A, k, W=W, target_sizes=rng.uniform(0.5, 2.0, k))
    # second call: fewer points, fewer blocks, 2D, unit weights, one empty block
    X2 = [rng.random(30001), rng.random(30001)]
    k2 = 37
    A2 = rng.integers(0, k2 - 1, 30001).astype(np.int32)
    got = compare(X2, A2, k2)
    assert got["empty_blocks"] == 1


def test_noalloc_stats_largest_k_and_limit():
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(8)
    n = 300000
    X = [rng.random(n).astype(np.float32), rng.random(n).astype(np.float32)]
    k = 65536
    A = rng.integers(0, k, n).astype(np.int32)
    compare(X, A, k, target_sizes=rng.uniform(0.5, 2.0, k))
    with pytest.raises(bkm.BkmError, match="no-allocation limit"):
        bkm.partition_stats_noalloc(cuda(X), torch.from_numpy(A).cuda(), k + 1)
