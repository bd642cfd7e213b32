"""Seeded synthetic point clouds (numpy PCG64), shared by tests and the benchmark.

This module only draws inputs.  It holds none of the partitioning arithmetic,
imports neither the GPU binding nor the oracle, and is the one piece both
sides of a parity test share.

The clouds stand in for the paper's meshes, which are not redistributable
here (Sec. 5.2 "Test Data"): uniform unit-square points for the random
geometric / Delaunay inputs, a refined-mesh mix of uniform and Gaussian
clusters for the adaptively refined 2D meshes, dense shells around spheres
for the 3D respiratory meshes, and a 1/r density with log-normal node weights
for the weighted 2.5D climate meshes.

Every generator returns a dict with
    X  : list of d contiguous 1-D arrays (SoA), float64 (float32 for C5)
    W  : float64 node weights or None (unit weights)
    k, eps, name
"""
import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n, d, seed, lo=0.0, hi=1.0):
    """n points uniform in [lo, hi]^d."""
    g = _rng(seed)
    return [g.uniform(lo, hi, n) for _ in range(d)]


def c1(seed=1, n=100_000):
    """2D, uniform in the unit square, unit weights, k=16, eps=0.03."""
    return dict(name="c1_uniform2d", X=uniform(n, 2, seed), W=None, k=16, eps=0.03)


def refined2d(n, seed, n_gauss=8):
    """70% uniform in [0,1]^2, 30% split evenly over n_gauss Gaussians with
    means uniform in [0.1,0.9]^2 and sigma log-uniform in [0.005, 0.05]
    (not clipped)."""
    g = _rng(seed)
    n_uni = int(round(0.7 * n))
    n_g = n - n_uni
    mu = g.uniform(0.1, 0.9, (n_gauss, 2))
    sig = np.exp(g.uniform(math.log(0.005), math.log(0.05), n_gauss))
    counts = np.full(n_gauss, n_g // n_gauss)
    counts[: n_g - counts.sum()] += 1
    x = np.empty(n)
    y = np.empty(n)
    x[:n_uni] = g.uniform(0.0, 1.0, n_uni)
    y[:n_uni] = g.uniform(0.0, 1.0, n_uni)
    o = n_uni
    for i in range(n_gauss):
        c = int(counts[i])
        x[o:o + c] = g.normal(mu[i, 0], sig[i], c)
        y[o:o + c] = g.normal(mu[i, 1], sig[i], c)
        o += c
    # interleave so that the input order carries no spatial structure
    p = g.permutation(n)
    return [np.ascontiguousarray(x[p]), np.ascontiguousarray(y[p])]


def c2(seed=2, n=16_000_000, k=1024):
    """2D refined-mesh cloud, unit weights, k=1024, eps=0.03."""
    return dict(name="c2_refined2d", X=refined2d(n, seed), W=None, k=k, eps=0.03)


def shells3d(n, seed, n_sph=16, box=(4.0, 1.0, 1.0), shell=0.05, p_out=0.1,
             chunk=1 << 22):
    """Points in a box, ten times denser within `shell` of n_sph random
    sphere surfaces (centers uniform in the box, radii uniform in [0.1, 0.5]):
    a uniform candidate is kept with probability 1 near a surface, else
    p_out."""
    g = _rng(seed)
    cen = np.stack([g.uniform(0.0, b, n_sph) for b in box], axis=1)
    rad = g.uniform(0.1, 0.5, n_sph)
    out = [np.empty(n) for _ in range(3)]
    have = 0
    while have < n:
        cand = [g.uniform(0.0, b, chunk) for b in box]
        u = g.uniform(0.0, 1.0, chunk)
        c32 = [c.astype(np.float32) for c in cand]
        near = np.zeros(chunk, dtype=bool)
        for s in range(n_sph):
            dx = c32[0] - np.float32(cen[s, 0])
            dy = c32[1] - np.float32(cen[s, 1])
            dz = c32[2] - np.float32(cen[s, 2])
            r = np.sqrt(dx * dx + dy * dy + dz * dz)
            near |= np.abs(r - np.float32(rad[s])) <= np.float32(shell)
        keep = near | (u < p_out)
        m = min(int(keep.sum()), n - have)
        idx = np.flatnonzero(keep)[:m]
        for j in range(3):
            out[j][have:have + m] = cand[j][idx]
        have += m
    return out


def c3(seed=3, n=64_000_000, k=4096):
    """3D, 4x1x1 box, 10x denser near 16 sphere surfaces, unit weights,
    k=4096, eps=0.03."""
    return dict(name="c3_shells3d", X=shells3d(n, seed), W=None, k=k, eps=0.03)


def radial2d_f32(n, seed, chunk=1 << 22):
    """FP32 points in [0,1]^2 with density proportional to 1/(r+0.01) around
    (0.5,0.5): r ~ U[0, sqrt(2)/2] kept with probability r/(r+0.01), theta
    uniform, points outside the square rejected."""
    g = _rng(seed)
    x = np.empty(n, dtype=np.float32)
    y = np.empty(n, dtype=np.float32)
    have = 0
    rmax = math.sqrt(2.0) / 2.0
    while have < n:
        r = g.uniform(0.0, rmax, chunk)
        acc = g.uniform(0.0, 1.0, chunk) < r / (r + 0.01)
        th = g.uniform(0.0, 2.0 * math.pi, chunk)
        px = 0.5 + r * np.cos(th)
        py = 0.5 + r * np.sin(th)
        keep = acc & (px >= 0.0) & (px <= 1.0) & (py >= 0.0) & (py <= 1.0)
        m = min(int(keep.sum()), n - have)
        idx = np.flatnonzero(keep)[:m]
        x[have:have + m] = px[idx]
        y[have:have + m] = py[idx]
        have += m
    return [x, y]


def c5(seed=5, n=250_000_000, k=16384):
    """2D FP32 radial cloud with log-normal(0, 0.5) FP64 node weights,
    k=16384, eps=0.03."""
    X = radial2d_f32(n, seed)
    W = _rng(seed + 1000).lognormal(0.0, 0.5, n)
    return dict(name="c5_radial2d_weighted", X=X, W=W, k=k, eps=0.03)


def gauss3d(n, seed, n_gauss=8):
    """3D: n_gauss Gaussian clusters in [0,1]^3, sigma log-uniform in
    [0.01, 0.1]."""
    g = _rng(seed)
    mu = g.uniform(0.0, 1.0, (n_gauss, 3))
    sig = np.exp(g.uniform(math.log(0.01), math.log(0.1), n_gauss))
    lab = g.integers(0, n_gauss, n)
    return [np.ascontiguousarray(g.normal(mu[lab, j], sig[lab])) for j in range(3)]


def c4(seed=4, count=256, n_lo=10_000, n_hi=2_000_000, k_lo=8, k_hi=512):
    """Batch of instances: n log-uniform in [n_lo, n_hi], k log-uniform in
    [k_lo, k_hi]; even ids 2D uniform, odd ids 3D Gaussian clusters."""
    g = _rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        k = int(round(math.exp(g.uniform(math.log(k_lo), math.log(k_hi)))))
        k = max(1, min(k, n))
        X = uniform(n, 2, seed * 100003 + i) if i % 2 == 0 else gauss3d(n, seed * 100003 + i)
        out.append(dict(name=f"c4_{i}", X=X, W=None, k=k, eps=0.03))
    return out


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def splitmix64(seed, n):
    """Random order keys for the random-sample initialization: outputs 0..n-1
    of splitmix64 seeded with `seed` (Steele, Lea, Flood, "Fast splittable
    pseudorandom number generators", OOPSLA 2014): output i mixes the state
    seed + (i+1) * 0x9E3779B97F4A7C15 (mod 2^64) with the 64-bit finaliser of
    shift-xors by 30, 27, 31 and multiplies by 0xBF58476D1CE4E5B9 and
    0x94D049BB133111EB.  Returns uint64[n]."""
    with np.errstate(over="ignore"):
        z = (np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
             + np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))
