"""Seeded synthetic inputs shared by tests, the smoke check and the benchmark.

This module only draws grids and test densities; it contains none of the
solver's arithmetic and imports nothing from the solver or the oracle.

Densities are sums of compact radial bumps A_i (1 - |x - c_i|^2/w_i^2)^p
(the paper's test family, Section 6, eq. Bepsilon, without the unit-integral
factor unless asked for), sampled on a uniform grid x = lo + i h.
"""
from __future__ import annotations

import numpy as np


def grid_spacing(n, lo=-1.0, hi=1.0):
    """Mesh widths of the uniform grid with n[i] nodes on [lo_i, hi_i]."""
    n = np.atleast_1d(np.asarray(n, dtype=np.int64))
    lo = np.broadcast_to(np.asarray(lo, np.float64), n.shape)
    hi = np.broadcast_to(np.asarray(hi, np.float64), n.shape)
    return (hi - lo) / (n - 1)


def node_coords(n, lo=-1.0, hi=1.0):
    """List of 1D coordinate arrays x_i = lo + i h, i = 0..n-1, one per axis."""
    n = np.atleast_1d(np.asarray(n, dtype=np.int64))
    lo = np.broadcast_to(np.asarray(lo, np.float64), n.shape)
    h = grid_spacing(n, lo, np.broadcast_to(np.asarray(hi, np.float64), n.shape))
    return [lo[a] + h[a] * np.arange(n[a], dtype=np.float64) for a in range(len(n))]


def bump_params(seed: int, d: int, count: int = 5):
    """Centres c ~ U[-0.5, 0.5]^d, widths w ~ U[0.2, 0.4], amplitudes A ~ N(0, 1), in that order."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, (count, d))
    w = rng.uniform(0.2, 0.4, count)
    a = rng.standard_normal(count)
    return c, w, a


def bump_sum(n, centers, widths, amps, p: int = 10, lo=-1.0, hi=1.0) -> np.ndarray:
    """rho(x) = sum_i A_i max(0, 1 - |x - c_i|^2 / w_i^2)^p on the grid (FP64)."""
    coords = node_coords(n, lo, hi)
    d = len(coords)
    mesh = np.meshgrid(*coords, indexing="ij")
    rho = np.zeros(mesh[0].shape)
    for c, w, a in zip(np.asarray(centers), np.asarray(widths), np.asarray(amps)):
        r2 = sum((mesh[k] - c[k]) ** 2 for k in range(d))
        t = np.maximum(0.0, 1.0 - r2 / (w * w))
        rho += a * t ** p
    return rho


def radial_bump(n, eps: float, p: int, center=None, gamma: float = 1.0, lo=-1.0, hi=1.0):
    """gamma (1 - |x - center|^2/eps^2)^p for |x - center| < eps, else 0."""
    n = np.atleast_1d(np.asarray(n, dtype=np.int64))
    d = len(n)
    center = np.zeros(d) if center is None else np.asarray(center, np.float64)
    return bump_sum(n, center[None, :], np.array([eps]), np.array([gamma]), p, lo, hi)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def workload_2d_single(n: int = 65):
    """2D, n x n on [-1,1]^2, rho = (1 - r^2/0.64)^8 for r < 0.8, centred, 4th order."""
    rho = radial_bump((n, n), 0.8, 8)
    h = grid_spacing((n, n))
    return rho, h, dict(eps=0.8, p=8, center=np.zeros(2), order=4)


def workload_bumps_3d(n: int, seed: int, p: int = 10):
    """3D, n^3 on [-1,1]^3, sum of 5 seeded compact bumps (C^9 for p = 10)."""
    c, w, a = bump_params(seed, 3)
    rho = bump_sum((n, n, n), c, w, a, p)
    h = grid_spacing((n, n, n))
    return rho, h, dict(centers=c, widths=w, amps=a, p=p)


def workload_bumps(n, seed: int, p: int = 10, scale=None):
    """Any-dimension bump sum on the box [-s, s] (s = scale per axis, default 1)."""
    n = np.atleast_1d(np.asarray(n, dtype=np.int64))
    d = len(n)
    s = np.ones(d) if scale is None else np.asarray(scale, np.float64)
    c, w, a = bump_params(seed, d)
    c = c * s
    w = w * float(np.min(s))
    rho = bump_sum(n, c, w, a, p, lo=-s, hi=s)
    h = grid_spacing(n, -s, s)
    return rho, h, dict(centers=c, widths=w, amps=a, p=p, lo=-s, hi=s)


def batched_problems(seed: int = 3, count: int = 64, nmin: int = 33, nmax: int = 193):
    """Independent 3D problems of uneven size: per axis n = round(exp(U(ln nmin, ln nmax))),
    box [-s_i, s_i] with s_i ~ U(0.5, 2), bump sum drawn from ``seed + 1000 + index``."""
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        n = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), 3))).astype(np.int64)
        s = rng.uniform(0.5, 2.0, 3)
        rho, h, meta = workload_bumps(n, seed + 1000 + b, scale=s)
        probs.append((rho, h, meta))
    return probs
