"""The seeded input generators themselves: the random order keys of the
random-sample initialization must be splitmix64's published outputs."""
from pathlib import Path

import numpy as np

from paper_1805_01208_amd import workloads

GOLDEN = Path(__file__).parent / "golden" / "splitmix64_vectors.txt"


def test_splitmix64_matches_published_outputs():
    rows = [ln.split() for ln in GOLDEN.read_text().splitlines()
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 2
    for row in rows:
        seed, want = int(row[0]), [int(v) for v in row[1:]]
        got = workloads.splitmix64(seed, len(want))
        assert got.dtype == np.uint64
        assert [int(v) for v in got] == want


def test_splitmix64_is_a_stream():
    """Output i depends on the seed and i alone (counter-based): a longer
    draw extends a shorter one, and seeds one gamma apart are shifted
    streams."""
    a = workloads.splitmix64(99, 1000)
    assert np.array_equal(workloads.splitmix64(99, 10), a[:10])
    b = workloads.splitmix64(99 + 0x9E3779B97F4A7C15, 999)
    assert np.array_equal(b, a[1:])
    assert len(np.unique(a)) == 1000
