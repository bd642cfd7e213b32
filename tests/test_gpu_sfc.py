"""GPU Hilbert bootstrap against the oracle: keys, stable sort permutation and
initial centers bit-exact (Alg. 2; Sec. 4.1)."""
import numpy as np
import pytest

import oracle
from gpu_common import cuda, torch, widened

pytestmark = pytest.mark.gpu

CASES = [
    # (d, dtype, n, k, order)
    (2, np.float64, 70001, 16, 16),
    (3, np.float64, 50003, 100, 16),
    (2, np.float32, 33333, 7, 31),
    (3, np.float32, 20000, 64, 21),
    (2, np.float64, 4000, 10, 3),    # coarse order: many equal keys, stability matters
    (3, np.float64, 1, 1, 16),
    (2, np.float64, 1000, 1000, 16),
]


@pytest.mark.parametrize("d,dtype,n,k,m", CASES)
def test_sfc_bootstrap_bit_exact(d, dtype, n, k, m):
    from paper_1805_01208_amd import bkm
    rng = np.random.default_rng(n + d)
    X = [rng.random(n).astype(dtype) * (4.0 if j == 0 else 1.0) for j in range(d)]
    print(f"case d={d} {np.dtype(dtype).name} n={n} k={k} m={m}", flush=True)
    C, perm, keys = bkm.init_centers_sfc(cuda(X), k, m)
    oc, operm, okeys = oracle.init_centers_sfc(widened(X), k, m)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), okeys)
    assert np.array_equal(perm.cpu().numpy().astype(np.int64), operm)
    assert np.array_equal(C.cpu().numpy(), oc)


def test_zero_extent():
    from paper_1805_01208_amd import bkm
    X = [np.full(3000, 0.3), np.full(3000, -2.0)]
    C, perm, keys = bkm.init_centers_sfc(cuda(X), 5, 16)
    assert torch.all(keys == 0)
    assert np.array_equal(perm.cpu().numpy(), np.arange(3000, dtype=np.int32))
    assert np.all(C.cpu().numpy() == [0.3, -2.0])


def test_non_finite_input_is_rejected():
    from paper_1805_01208_amd import bkm
    x = np.random.default_rng(0).random(500)
    x[17] = np.nan
    with pytest.raises(bkm.BkmError) as e:
        bkm.init_centers_sfc(cuda([x, x.copy()]), 4, 16)
    assert e.value.code == bkm.BKM_EDATA
