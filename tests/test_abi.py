"""The C-ABI library loads and exports every entry point include/bkm.h
declares; argument errors are reported without touching a GPU."""
import ctypes as C
import os
import subprocess
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bkm.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bkm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def bkm():
    from paper_1805_01208_amd import bkm as b
    if not os.path.exists(b.LIB_PATH):
        from paper_1805_01208_amd import build
        build.build()
    return b


def test_header_declares_the_boundary():
    names = declared()
    for f in ("bkm_init_centers_sfc", "bkm_balanced_kmeans", "bkm_balanced_kmeans_batched",
              "bkm_partition_stats", "bkm_last_error"):
        assert f in names


def test_every_declared_symbol_is_exported(bkm):
    L = bkm.lib()
    for name in declared():
        assert hasattr(L, name), name
    assert set(bkm.FUNCTIONS) == set(declared())


def test_struct_layouts_match_header(bkm, tmp_path):
    """Size and every field offset of the binding's structs against the
    header, compiled by the host C compiler."""
    structs = {"bkm_points": bkm.Points, "bkm_params": bkm.Params, "bkm_info": bkm.Info,
               "bkm_stats": bkm.Stats, "bkm_graph_stats": bkm.GraphStats,
               "bkm_knn_info": bkm.KnnInfo, "bkm_tune_result": bkm.TuneResult}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "bkm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_default_params(bkm):
    p = bkm.default_params(16)
    assert (p.k, p.max_iter, p.max_balance_iter, p.hilbert_order) == (16, 50, 20, 16)
    assert p.precision == bkm.PREC_F32_RECHECK and p.use_bounds == 1
    assert p.epsilon == 0.03 and p.delta_threshold < 0 and p.recheck_rel_gap == 1e-5
    assert (p.sample_init, p.sample_start, p.seed, p.sample_keys) == (0, 0, 0, None)
    assert p.target_sizes is None and p.erosion == 1


def _pts(bkm, n=100, d=2, dtype=1):
    p = bkm.Points()
    p.n, p.d, p.dtype = n, d, dtype
    for j in range(3):
        p.coords[j] = 0x1000 if j < d else None  # never dereferenced: rejected first
    p.weights = None
    return p


@pytest.mark.parametrize("mutate,needle", [
    (lambda p, q: setattr(p, "d", 4), "d = 4"),
    (lambda p, q: setattr(p, "n", 0), "n = 0"),
    (lambda p, q: setattr(p, "dtype", 7), "dtype"),
    (lambda p, q: setattr(q, "k", 0), "k = 0"),
    (lambda p, q: setattr(q, "k", 101), "k = 101"),
    (lambda p, q: setattr(q, "epsilon", -0.5), "epsilon"),
    (lambda p, q: setattr(q, "epsilon", float("nan")), "epsilon"),
    (lambda p, q: setattr(q, "max_iter", 0), "max_iter"),
    (lambda p, q: setattr(q, "hilbert_order", 32), "hilbert_order"),
    (lambda p, q: setattr(q, "precision", 5), "precision"),
    (lambda p, q: setattr(q, "tile_points", 300), "tile_points"),
    (lambda p, q: setattr(q, "recheck_rel_gap", -1.0), "recheck_rel_gap"),
    (lambda p, q: (setattr(q, "sample_init", 1), setattr(q, "sample_start", -1)), "sample_start"),
    (lambda p, q: setattr(q, "erosion", 2), "erosion"),
])
def test_invalid_arguments(bkm, mutate, needle):
    L = bkm.lib()
    p = _pts(bkm)
    q = bkm.default_params(10)
    mutate(p, q)
    rc = L.bkm_balanced_kmeans(C.byref(p), C.byref(q), None, C.c_void_p(0x2000),
                               C.c_void_p(0x3000), None, None, None, None)
    assert rc == bkm.BKM_EINVAL
    assert needle in L.bkm_last_error().decode()


def test_3d_order_limit_and_null_outputs(bkm):
    L = bkm.lib()
    p = _pts(bkm, d=3)
    rc = L.bkm_init_centers_sfc(C.byref(p), 4, 22, C.c_void_p(0x2000), None, None, None)
    assert rc == bkm.BKM_EINVAL and "hilbert_order" in L.bkm_last_error().decode()
    rc = L.bkm_init_centers_sfc(C.byref(p), 4, 16, None, None, None, None)
    assert rc == bkm.BKM_EINVAL
    q = bkm.default_params(4)
    rc = L.bkm_balanced_kmeans(C.byref(p), C.byref(q), None, None, None, None, None, None, None)
    assert rc == bkm.BKM_EINVAL
    rc = L.bkm_partition_stats(None, None, 4, 0.03, None, None, None, None, None)
    assert rc == bkm.BKM_EINVAL
    rc = L.bkm_assign_sweeps(C.byref(p), 4, 0, None, None, 0, 1, 0, None, None, None, None)
    assert rc == bkm.BKM_EINVAL


def test_graph_argument_errors(bkm):
    """Rejected on the host before any device work."""
    L = bkm.lib()
    p = _pts(bkm, n=10)
    assert L.bkm_knn(C.byref(p), 0, C.c_void_p(0x2000), None, None, None) == bkm.BKM_EINVAL
    assert L.bkm_knn(C.byref(p), 17, C.c_void_p(0x2000), None, None, None) == bkm.BKM_EINVAL
    assert L.bkm_knn(C.byref(p), 10, C.c_void_p(0x2000), None, None, None) == bkm.BKM_EINVAL
    assert "knn + 1" in L.bkm_last_error().decode()
    assert L.bkm_knn(C.byref(p), 4, None, None, None, None) == bkm.BKM_EINVAL
    assert L.bkm_knn_graph(1, 1, C.c_void_p(0x2000), None, C.c_void_p(0x3000),
                           C.c_void_p(0x4000), None, None) == bkm.BKM_EINVAL
    assert L.bkm_knn_graph(10, 10, C.c_void_p(0x2000), None, C.c_void_p(0x3000),
                           C.c_void_p(0x4000), None, None) == bkm.BKM_EINVAL
    st = bkm.GraphStats()
    assert L.bkm_graph_metrics(10, 5, None, None, None, 2, None, None, None, C.byref(st),
                               None) == bkm.BKM_EINVAL
    assert L.bkm_graph_metrics(10, -1, C.c_void_p(0x2000), C.c_void_p(0x3000),
                               C.c_void_p(0x4000), 2, None, None, None, C.byref(st),
                               None) == bkm.BKM_EINVAL
    assert L.bkm_graph_metrics(10, 5, C.c_void_p(0x2000), C.c_void_p(0x3000),
                               C.c_void_p(0x4000), 0, None, None, None, C.byref(st),
                               None) == bkm.BKM_EINVAL


def test_batched_argument_errors(bkm):
    """Checked per instance before any device work; the message names the instance."""
    L = bkm.lib()
    pts = (bkm.Points * 3)(_pts(bkm), _pts(bkm, d=3), _pts(bkm))
    prm = (bkm.Params * 3)(bkm.default_params(10), bkm.default_params(10), bkm.default_params(10))
    outs = (C.c_void_p * 3)(0x2000, 0x2000, 0x2000)
    cen = (C.c_void_p * 3)(0x3000, 0x3000, 0x3000)
    assert L.bkm_balanced_kmeans_batched(pts, prm, 0, outs, cen, None, None) == bkm.BKM_EINVAL
    assert "count" in L.bkm_last_error().decode()
    assert L.bkm_balanced_kmeans_batched(None, prm, 3, outs, cen, None, None) == bkm.BKM_EINVAL
    prm[1].k = 0
    assert L.bkm_balanced_kmeans_batched(pts, prm, 3, outs, cen, None, None) == bkm.BKM_EINVAL
    assert L.bkm_last_error().decode().startswith("instance 1: k = 0")
    prm[1].k = 10
    cen[2] = None
    assert L.bkm_balanced_kmeans_batched(pts, prm, 3, outs, cen, None, None) == bkm.BKM_EINVAL
    assert L.bkm_last_error().decode().startswith("instance 2:")
    cen[2] = 0x3000
    prm[0].sample_init = 1
    assert L.bkm_balanced_kmeans_batched(pts, prm, 3, outs, cen, None, None) == bkm.BKM_EINVAL
    assert L.bkm_last_error().decode().startswith("instance 0: sample_init")


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1805_01208_amd import bkm as b
    monkeypatch.setattr(b, "_LIB", None)
    monkeypatch.setattr(b, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        b.lib()
