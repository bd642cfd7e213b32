#!/usr/bin/env python3
"""Balanced k-means on one MI355X: points assigned per second per sweep.

One step = one whole bkm_balanced_kmeans call on the resident synthetic cloud:
Hilbert bootstrap (bounding box, keys, radix sort, permutation, tiles,
initial centers) and every AssignAndBalance round until convergence or
max_iter (sweeps with their balance tests, block boxes, center moves).
value = n * (sweeps made in the step) / (step wall time), averaged over the
timed steps, with the FP32-screen + FP64-recheck sweep.  The plain FP64 sweep
on the same cloud is timed beside it.

The roofline figure is for the dominant kernel, the assignment sweep: its
device time comes from HIP events the library records around every sweep
launch on the call's stream; its algorithmic bytes come from the run's
visit counters (see algorithmic_bytes).  The CPU baseline is the plain FP64
oracle timed on a bounded random sample of the same cloud.

Prints one JSON line.

With --graph it measures the graph-quality evaluation instead (Sec. 2 block
measures on a k-nearest-neighbour graph of the cloud): one step = exact
K-nearest-neighbour lists, their undirected CSR graph, and the edge cut,
communication volume and block diameter bounds of the cloud's balanced
k-means partition (computed once, untimed).  value = points per second
through the step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "points assigned/s per balanced k-means sweep, FP32+recheck vs FP64, ε=0.03"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(info, d, precision, weighted):
    """Bytes a sweep must move, from the run's visit counters.

    every visit: block id (4) + stored upper and lower bound (4 + 4), read;
    evaluated:   working coordinates read (FP32 screen: one packed fixed-point
                 word, 4 bytes in 2D and 8 in 3D; plain FP64: 8d), both bounds
                 written (8);
    changed:     block id written (4), the weight (8, weighted) read for the
                 block-weight transfer;
    rechecked:   FP64 coordinates read (8d);
    per 64-point group: its common-block flag written (4)."""
    visits = info["evaluated"] + info["skipped"]
    f32 = precision == "f32_recheck"
    b = 12 * visits + 4 * visits / 64
    b += info["evaluated"] * ((4 if d == 2 else 8) if f32 else 8 * d) + info["evaluated"] * 8
    b += info["changed"] * (4 + (8 if weighted else 0))
    if f32:
        b += info["rechecked"] * 8 * d
    return b


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_c3_hbm_traffic.txt")
SWEEP_SOURCES = [os.path.join(ROOT, "paper_1805_01208_amd", "csrc", f)
                 for f in ("bkm_sweep.hip", "bkm_internal.h")]


def sweep_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, tile):
    """HBM bytes per sweep launch from the committed counter summary (memory-side
    requests by size), as (total, read, write), or None when it is missing, was
    taken on another workload, or the sweep kernel's source has changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split(":", 1) for line in fh if ":" in line and not line.startswith(" "))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sweep_source_digest") != sweep_source_digest():
        return None
    if kv.get("workload") != workload or kv.get("tile_points") != str(tile):
        return None
    try:
        return (float(kv["hbm_bytes_per_launch"]), float(kv["read_bytes_per_launch"]),
                float(kv["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def copy_calibration(torch):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters to bytes."""
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                           "launches": 3}}), flush=True)


def make_workload(name, n=None):
    from paper_1805_01208_amd import workloads
    kw = {} if n is None else {"n": n}
    return workloads.CONFIGS[name](**kw)


def cpu_baseline(cfg, budget_s):
    """The oracle's sweep (brute-force argmin over all k centers, block
    weights, balance test) on a random sample of the workload."""
    import numpy as np
    import oracle
    X = cfg["X"]
    W = cfg["W"]
    n = len(X[0])
    k = cfg["k"]
    rng = np.random.default_rng(12345)

    def sweep(m):
        idx = np.sort(rng.choice(n, size=m, replace=False))
        Xs = [np.asarray(x[idx], dtype=np.float64) for x in X]
        Ws = None if W is None else np.asarray(W[idx])
        kk = min(k, m)
        C, _, _ = oracle.init_centers_sfc(Xs, kk, 16)
        I = np.ones(kk)
        t0 = time.perf_counter()
        A, _, _ = oracle.assign(Xs, C, I)
        bw = oracle.block_weights(A, Ws, kk)
        tw = oracle.total_weight(m, Ws)
        oracle.balance_step(bw, len(X), oracle.lmax(m, kk, cfg["eps"], Ws), tw / kk, I)
        return time.perf_counter() - t0

    m0 = min(n, 4096)
    t0 = sweep(m0)
    m = int(min(n, max(m0, m0 * budget_s / max(t0, 1e-6))))
    t = sweep(m)
    return dict(value=m / t, unit="points/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"{m} random points of the workload, k={min(k, m)} SFC centers of the "
                       f"sample, one oracle sweep (FP64 brute-force argmin over all centers, "
                       f"block weights, balance test): {t:.2f} s")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_pruned(cfg, budget_s):
    """The pruned FP64 CPU baseline (Hamerly bounds + bounding-box candidates,
    OpenMP; equal to the oracle bit for bit) running the whole balanced k-means
    on a random sample of the workload with k scaled to keep the mean block
    size; points per second per sweep (sample size x sweeps / time in sweeps),
    median of 5 runs, on all host threads and on one thread."""
    import numpy as np
    import baseline
    import oracle
    X = cfg["X"]
    n = len(X[0])
    k = cfg["k"]
    rng = np.random.default_rng(2468)

    def sample(m):
        idx = np.sort(rng.choice(n, size=m, replace=False))
        Xs = [np.asarray(x[idx], dtype=np.float64) for x in X]
        ks = max(1, min(m, int(round(k * m / n))))
        C0, _, _ = oracle.init_centers_sfc(Xs, ks, 16)
        return Xs, ks, C0

    def runs(m, reps):
        Xs, ks, C0 = sample(m)
        vals, last = [], None
        for _ in range(reps):
            last = baseline.balanced_kmeans(Xs, ks, cfg["eps"], C0)["info"]
            vals.append(m * last["sweeps"] / max(last["sweep_seconds"], 1e-9))
        return float(np.median(vals)), ks, last

    out = {}
    all_threads = baseline.num_threads()
    for label, threads in (("all_threads", all_threads), ("one_thread", 1)):
        baseline.set_threads(threads)
        m0 = min(n, 100_000)
        _, _, pilot = runs(m0, 1)
        per_run = budget_s / 10.0
        m = int(min(n, max(m0, m0 * per_run / max(pilot["total_seconds"], 1e-6))))
        v, ks, last = runs(m, 5)
        out[label] = {"value": v, "unit": "points/s", "cores": threads,
                      "sample": f"{m} random points, k={ks}, a whole balanced k-means run "
                                f"({last['sweeps']} sweeps, skip {last['skipped'] / max(1, last['skipped'] + last['evaluated']):.3f}), "
                                f"median of 5"}
    baseline.set_threads(all_threads)
    out["kind"] = "pruned FP64 (Hamerly + box candidates), equal to the oracle"
    out["cpu_model"] = cpu_model()
    return out


def run_steps(bkm, torch, X, W, cfg, precision, steps, warmup, max_iter, tile=0, sup=0,
              extra=None):
    n = X[0].numel()
    k = cfg["k"]
    dev = X[0].device
    out = dict(A=torch.empty(n, dtype=torch.int32, device=dev),
               centers=torch.empty((k, len(X)), dtype=torch.float64, device=dev),
               influence=torch.empty(k, dtype=torch.float64, device=dev),
               block_weights=torch.empty(k, dtype=torch.float64, device=dev))

    extra = extra or {}

    def one():
        return bkm.balanced_kmeans(X, k, W=W, eps=cfg["eps"], max_iter=max_iter,
                                   precision=precision, tile_points=tile, super_tiles=sup,
                                   timing=True, out=out, **extra)

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(one()["info"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tot = {key: sum(i[key] for i in infos) for key in infos[0]}
    return wall, tot, infos[-1], out


def error_vs_oracle(bkm, torch, X, Xh, W, cfg, out, samples=20000):
    """Error of the last timed run against the oracle: its centers against
    the exact weighted means of its blocks (all points, on the host), and one
    fresh FP32+recheck sweep on its final centers and influence against the
    oracle's brute-force argmin on a random sample of points (mismatches
    outside and inside the 1e-12 tie gap)."""
    import numpy as np
    import oracle
    k = cfg["k"]
    A = out["A"].cpu().numpy()
    C = out["centers"].cpu().numpy()
    Wh = cfg["W"]
    wsum = np.bincount(A, weights=Wh, minlength=k) if Wh is not None else \
        np.bincount(A, minlength=k).astype(np.float64)
    ne = wsum > 0
    err = 0.0
    for j, x in enumerate(Xh):
        xs = np.asarray(x, dtype=np.float64)
        ref = np.bincount(A, weights=xs if Wh is None else Wh * xs, minlength=k)[ne] / wsum[ne]
        scale = max(float(np.max(np.abs(ref))), float(xs.max() - xs.min()))
        err = max(err, float(np.max(np.abs(C[ne, j] - ref))) / scale)
    I = out["influence"].cpu().numpy()
    As, _, _ = bkm.assign_sweeps(X, torch.from_numpy(C[None]), torch.from_numpy(I[None]),
                                 precision="f32_recheck")
    rng = np.random.default_rng(4242)
    idx = np.sort(rng.choice(len(A), size=min(samples, len(A)), replace=False))
    Ao, best, second = oracle.assign([np.asarray(x[idx], dtype=np.float64) for x in Xh], C, I)
    bad = As[0].cpu().numpy()[idx] != Ao
    tie = (second - best) / np.maximum(best, 1e-300) < 1e-12
    return {"sample_points": int(len(idx)), "assignment_mismatches": int(np.sum(bad & ~tie)),
            "mismatches_at_ties": int(np.sum(bad & tie)), "max_center_rel_err": err,
            "block_weights_exact": bool(Wh is not None or np.array_equal(
                out["block_weights"].cpu().numpy(), wsum))}


def extra_workloads(bkm, torch):
    """The other workloads, one figure each (points assigned per second per
    sweep over whole calls, inputs resident): C2 with the plain FP64 sweep,
    the 256-instance batch C4 in one batched call, and C5 (250M weighted
    FP32 points).  Tilings from the autotuner."""
    import numpy as np
    out = {}

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [fn() for _ in range(steps)]
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, res[-1]

    cfg = make_workload("c2")
    X = [torch.from_numpy(x).cuda() for x in cfg["X"]]
    n = len(cfg["X"][0])
    dt, g = timed(lambda: bkm.balanced_kmeans(X, cfg["k"], eps=cfg["eps"], precision="f64",
                                              timing=True), 3, 1)
    i = g["info"]
    out["c2_refined2d_fp64"] = {"value": n * i["sweeps"] / dt, "unit": "points/s",
                                "ms_per_call": 1e3 * dt, "sweeps": i["sweeps"],
                                "avg_sweep_us": 1e3 * i["sweep_ms"] / i["sweeps"],
                                "n": n, "k": cfg["k"], "precision": "f64"}
    del X
    print(f"[bench] c2 fp64: {out['c2_refined2d_fp64']}", file=sys.stderr, flush=True)

    cfgs = make_workload("c4")
    insts = [([torch.from_numpy(x).cuda() for x in c["X"]], c["k"]) for c in cfgs]
    npts = sum(len(c["X"][0]) for c in cfgs)
    dt, (res, rc) = timed(lambda: bkm.balanced_kmeans_batched(insts), 2, 1)
    sweeps = sum(o["info"]["sweeps"] for o in res)
    pts_sweeps = sum(len(c["X"][0]) * o["info"]["sweeps"] for c, o in zip(cfgs, res))
    out["c4_batched"] = {"value": pts_sweeps / dt, "unit": "points/s", "ms_per_call": 1e3 * dt,
                         "instances": len(cfgs), "points": npts, "sweeps": sweeps,
                         "return_code": rc, "precision": "f32_recheck"}
    del insts
    print(f"[bench] c4 batched: {out['c4_batched']}", file=sys.stderr, flush=True)

    cfg = make_workload("c5")
    X = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in cfg["X"]]
    W = torch.from_numpy(cfg["W"]).cuda()
    n = len(cfg["X"][0])
    dt, g = timed(lambda: bkm.balanced_kmeans(X, cfg["k"], W=W, eps=cfg["eps"], timing=True), 2, 1)
    i = g["info"]
    out["c5_radial2d_weighted"] = {"value": n * i["sweeps"] / dt, "unit": "points/s",
                                   "ms_per_call": 1e3 * dt, "sweeps": i["sweeps"],
                                   "avg_sweep_us": 1e3 * i["sweep_ms"] / i["sweeps"],
                                   "n": n, "k": cfg["k"], "precision": "f32_recheck",
                                   "balanced": i["balanced"]}
    print(f"[bench] c5: {out['c5_radial2d_weighted']}", file=sys.stderr, flush=True)
    return out


FP64_PEAK_TFLOPS = 78.6


def graph_cpu_baseline(cfg, K, budget_s):
    """The oracle's brute-force K nearest neighbours of random query points
    over the whole cloud (the dominant part of the evaluation)."""
    import numpy as np
    import oracle
    X = [np.asarray(x, dtype=np.float64) for x in cfg["X"]]
    n = len(X[0])
    rng = np.random.default_rng(777)
    q0 = 64
    while True:   # grow the pilot until it is long enough to time
        t0 = time.perf_counter()
        oracle.knn_of(X, K, rng.choice(n, q0, replace=False))
        t = time.perf_counter() - t0
        if t >= 0.1 * budget_s or q0 >= n:
            break
        q0 = min(n, 4 * q0)
    q = int(min(n, max(q0, q0 * budget_s / max(t, 1e-6))))
    t0 = time.perf_counter()
    oracle.knn_of(X, K, rng.choice(n, q, replace=False))
    t = time.perf_counter() - t0
    return dict(value=q / t, unit="points/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"exact {K}-NN lists of {q} random query points by FP64 brute force over "
                       f"all {n} points: {t:.2f} s (graph and metrics not included)")


def graph_bench(args, torch, bkm, cfg, X):
    """Steps of the graph-quality evaluation on the resident cloud."""
    n, d, k, K = X[0].numel(), len(X), cfg["k"], args.knn
    part = bkm.balanced_kmeans(X, k, eps=cfg["eps"], max_iter=args.max_iter)
    A = part["A"]

    def one():
        nbr, kinfo = bkm.knn(X, K, order=True)
        rp, col = bkm.knn_graph(nbr, kinfo["order"])
        m = bkm.graph_metrics(rp, col, A, k)
        return kinfo, m, col.numel()

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res.append(one())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    search_s = sum(r[0]["search_ms"] for r in res) / 1e3 / args.steps
    layout_s = sum(r[0]["layout_ms"] for r in res) / 1e3 / args.steps
    pairs = res[-1][0]["group_visits"] * 64 * 64
    flops = pairs * (3 * d - 1)   # FP64 subtractions, squares and additions per pair
    achieved = flops / search_s / 1e12
    m, nnz = res[-1][1], res[-1][2]
    line = {
        "metric": f"points/s through exact {K}-NN graph + partition quality metrics",
        "value": n * args.steps / wall,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"] + "_knn_graph", "n": n, "d": d, "knn": K, "k": k},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_knn", "avg_search_ms": search_s * 1e3,
                     "pairs_per_launch": pairs, "flops_per_pair": 3 * d - 1},
        "layout_ms": layout_s * 1e3,
        "pairs_per_point": pairs / n,
        "graph": {"nnz": nnz, "edge_cut": m["edge_cut"], "max_comm": m["max_comm"],
                  "total_comm": m["total_comm"], "max_diameter": m["max_diameter"],
                  "disconnected_blocks": m["disconnected_blocks"],
                  "harmonic_diameter": m["harmonic_diameter"], "bfs_levels": m["bfs_levels"],
                  "exact_blocks": m["exact_blocks"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = graph_cpu_baseline(cfg, K, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--n", type=int, default=None, help="override the workload size")
    ap.add_argument("--max-iter", type=int, default=50)
    ap.add_argument("--tile", type=int, default=0,
                    help="points per tile (0: the library's autotuner, -1: the n/k rule)")
    ap.add_argument("--super", type=int, default=0, help="tiles per super-tile (0: tuned/default)")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-check", action="store_true",
                    help="skip the check against the oracle (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads' figures (C2 plain FP64, C4 batched, C5)")
    ap.add_argument("--graph", action="store_true",
                    help="measure the graph-quality evaluation instead of the partitioner")
    ap.add_argument("--knn", type=int, default=6, help="neighbours per point (--graph)")
    ap.add_argument("--sample-init", action="store_true",
                    help="start every run with the random-sample rounds (seed 1)")
    ap.add_argument("--targets", action="store_true",
                    help="non-uniform target block sizes: k log-normal(0, 0.5) relative sizes, seed 9")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU sharding; it is described as a design only).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    from paper_1805_01208_amd import bkm

    t_gen = time.perf_counter()
    cfg = make_workload(args.config, args.n)
    gen_s = time.perf_counter() - t_gen
    Xh = cfg["X"]
    d = len(Xh)
    n = len(Xh[0])
    print(f"[bench] {cfg['name']} n={n} d={d} k={cfg['k']} generated in {gen_s:.1f} s",
          file=sys.stderr, flush=True)
    X = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in Xh]
    W = None if cfg["W"] is None else torch.from_numpy(cfg["W"]).cuda()
    weighted = W is not None
    torch.cuda.synchronize()
    if args.graph:
        graph_bench(args, torch, bkm, cfg, X)
        return

    # the tiling: the autotuner's choice (measured here once, before the timed
    # steps, or taken from its cache), unless fixed on the command line
    tune = None
    tile, sup = args.tile, args.super
    if tile == 0:
        t_tune = time.perf_counter()
        tune = bkm.autotune(X, cfg["k"], W=W, precision="f32_recheck", super_tiles=sup)
        tune["seconds"] = time.perf_counter() - t_tune
        print(f"[bench] autotuned tiling: {tune}", file=sys.stderr, flush=True)
        tile, sup = tune["tile_points"], tune["super_tiles"]
    elif tile < 0:
        tile = 1024 if n / cfg["k"] >= 2048 else 512 if n / cfg["k"] >= 512 else 256
    sup = sup or 16

    extra = {}
    if args.sample_init:
        extra.update(sample_init=True, seed=1)
    if args.targets:
        extra["target_sizes"] = torch.from_numpy(
            np.random.default_rng(9).lognormal(0.0, 0.5, cfg["k"])).cuda()
    wall, tot, last, outs = run_steps(bkm, torch, X, W, cfg, "f32_recheck", args.steps,
                                      args.warmup, args.max_iter, tile, sup, extra)
    sweeps = tot["sweeps"]
    value = n * sweeps / wall
    ms_per_step = 1e3 * wall / args.steps
    print(f"[bench] f32_recheck: {ms_per_step:.2f} ms/step, {sweeps / args.steps:.1f} sweeps/step",
          file=sys.stderr, flush=True)

    fp64 = None
    if args.fp64_steps > 0:
        wall64, tot64, _, _ = run_steps(bkm, torch, X, W, cfg, "f64", args.fp64_steps, 1,
                                     args.max_iter, tile, sup, extra)
        sweep64_s = tot64["sweep_ms"] / 1e3 / tot64["sweeps"]
        algo64 = algorithmic_bytes(tot64, d, "f64", weighted) / tot64["sweeps"]
        fp64 = {"value": n * tot64["sweeps"] / wall64, "ms_per_step": 1e3 * wall64 / args.fp64_steps,
                "sweeps_per_step": tot64["sweeps"] / args.fp64_steps,
                "avg_sweep_us": sweep64_s * 1e6, "sweep_gbs": algo64 / sweep64_s / 1e9}
        print(f"[bench] f64: {fp64['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)

    sweep_s = tot["sweep_ms"] / 1e3 / sweeps
    algo = algorithmic_bytes(tot, d, "f32_recheck", weighted) / sweeps
    achieved = algo / sweep_s / 1e9
    # the committed counters are for the default run only
    traffic = None if (args.sample_init or args.targets) else measured_traffic(cfg["name"], tile)

    visits = tot["evaluated"] + tot["skipped"]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32_screen+f64_recheck",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "d": d, "k": cfg["k"], "eps": cfg["eps"],
                   "weighted": weighted, "precision": "f32_recheck", "max_iter": args.max_iter,
                   "max_balance_iter": 20, "hilbert_order": 16, "tile_points": tile,
                   "super_tiles": sup, "sample_init": bool(args.sample_init),
                   "target_sizes": "lognormal(0,0.5), seed 9" if args.targets else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic[0],
                     "traffic_read": None if traffic is None else traffic[1],
                     "traffic_write": None if traffic is None else traffic[2],
                     "traffic_frac": None if traffic is None else
                     traffic[0] / sweep_s / 1e9 / HBM_PEAK_GBS,
                     "kernel": "k_sweep", "avg_sweep_us": sweep_s * 1e6,
                     "algorithmic_bytes_per_launch": algo},
        "sweeps_per_step": sweeps / args.steps,
        "sample_sweeps_per_step": tot["sample_sweeps"] / args.steps,   # not counted in value
        "rounds_per_step": tot["rounds"] / args.steps,
        "skip_frac": tot["skipped"] / visits,
        "recheck_frac_of_evaluated": tot["rechecked"] / max(1, tot["evaluated"]),
        "candidates_per_evaluated": tot["candidate_evals"] / max(1, tot["evaluated"]),
        "kernel_ms_per_step": {kk: tot[kk] / args.steps for kk in
                               ("cand_ms", "sweep_ms", "balance_ms", "boxes_ms", "move_ms",
                                "bootstrap_ms", "total_ms")},
        "balanced": last["balanced"],
        "imbalance": last["imbalance"],
        "autotune": tune,
        "error_vs_oracle": None if args.no_error_check else
        error_vs_oracle(bkm, torch, X, Xh, W, cfg, outs),
    }
    if fp64 is not None:
        line["fp64_plain"] = fp64
        line["speedup_vs_fp64"] = value / fp64["value"]
        line["sweep_speedup_vs_fp64"] = fp64["avg_sweep_us"] / (sweep_s * 1e6)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
        line["cpu_baseline"]["cpu_model"] = cpu_model()
        if W is None:
            line["cpu_pruned"] = cpu_pruned(cfg, args.cpu_seconds)
    if not args.no_extras and args.config == "c3" and args.n is None:
        del X, W, outs
        torch.cuda.empty_cache()
        line["other_workloads"] = extra_workloads(bkm, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
