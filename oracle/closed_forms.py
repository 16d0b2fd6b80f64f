"""Exact free-space potentials of compact radial test densities (oracle pins).

TEST INFRASTRUCTURE ONLY.

The paper's test densities (Section 6, eq. Bepsilon) are translates of
rho(x) = gamma (1 - |x/eps|^2)^p for |x| <= eps, 0 outside, and it notes
that the potential of such a function can be written in closed form.  The
formulas below follow from radial symmetry and Gauss's theorem applied to
Delta phi = rho with phi = G * rho:

2D, with t = 1 - r^2/eps^2 and Q = pi eps^2 / (p + 1) (unit gamma):
    phi(r) = Q/(2 pi) log r                                    r >= eps
    phi(r) = Q/(2 pi) log eps - eps^2/(4 (p+1)) sum_{k=1}^{p+1} t^k / k   r < eps

3D, with Q = 4 pi int_0^eps rho(s) s^2 ds:
    phi(r) = -Q / (4 pi r)                                     r >= eps
    phi(r) = -(1/r) int_0^r rho(s) s^2 ds - eps^2/(2 (p+1)) t^(p+1)      r < eps

The inner integral is a polynomial of degree 2p+2 in s, integrated exactly
by Gauss-Legendre with p+2 (or more) nodes.  ``gamma`` scales everything
linearly (gamma = 1 gives the raw bump used by the synthetic workloads).
"""
from __future__ import annotations

import math

import numpy as np


def unit_gamma(d: int, eps: float, p: int) -> float:
    """gamma such that gamma (1 - |x/eps|^2)^p has unit integral in R^d."""
    if d == 1:
        # int_{-eps}^{eps} (1 - x^2/eps^2)^p dx = eps * B(1/2, p+1)
        m = eps * math.gamma(0.5) * math.gamma(p + 1) / math.gamma(p + 1.5)
    elif d == 2:
        m = math.pi * eps * eps / (p + 1)
    elif d == 3:
        m = 4.0 * math.pi * eps ** 3 * math.gamma(1.5) * math.gamma(p + 1) / (
            2.0 * math.gamma(p + 2.5)
        )
    else:
        raise ValueError("d must be 1, 2 or 3")
    return 1.0 / m


def radial_potential(d: int, r, eps: float, p: int, gamma: float = 1.0) -> np.ndarray:
    """phi(r) for rho = gamma (1 - r^2/eps^2)^p on r < eps (2D or 3D)."""
    r = np.asarray(r, dtype=np.float64)
    out = np.empty_like(r)
    inside = r < eps
    t = np.where(inside, 1.0 - (r * r) / (eps * eps), 0.0)
    if d == 2:
        Q = math.pi * eps * eps / (p + 1)
        rr = np.where(inside, 1.0, r)
        out[~inside] = Q / (2.0 * math.pi) * np.log(rr[~inside])
        s = np.zeros_like(r)
        tk = np.ones_like(r)
        for k in range(1, p + 2):
            tk = tk * t
            s = s + tk / k
        val_in = Q / (2.0 * math.pi) * math.log(eps) - eps * eps / (4.0 * (p + 1)) * s
        out[inside] = val_in[inside]
        return gamma * out
    if d == 3:
        Q = 4.0 * math.pi * eps ** 3 * math.gamma(1.5) * math.gamma(p + 1) / (
            2.0 * math.gamma(p + 2.5)
        )
        rr = np.where(inside, 1.0, r)
        out[~inside] = -Q / (4.0 * math.pi * rr[~inside])
        nodes, weights = np.polynomial.legendre.leggauss(p + 4)
        ri = r[inside]
        # int_0^r (1 - s^2/eps^2)^p s^2 ds with s = r (x + 1)/2
        s = 0.5 * ri[:, None] * (nodes[None, :] + 1.0)
        f = (1.0 - s * s / (eps * eps)) ** p * s * s
        integ = 0.5 * ri * (f @ weights)
        val = np.empty_like(ri)
        pos = ri > 0
        val[pos] = -integ[pos] / ri[pos]
        val[~pos] = 0.0  # limit r -> 0 of (1/r) int_0^r rho s^2 ds is 0
        val = val - eps * eps / (2.0 * (p + 1)) * t[inside] ** (p + 1)
        out[inside] = val
        return gamma * out
    raise ValueError("closed forms provided for d = 2 and 3")


def bump_sum_potential(points: np.ndarray, centers, widths, amps, p: int) -> np.ndarray:
    """Potential of sum_i A_i (1 - |x - c_i|^2 / w_i^2)^p at ``points`` (shape (..., d))."""
    points = np.asarray(points, dtype=np.float64)
    d = points.shape[-1]
    out = np.zeros(points.shape[:-1])
    for c, w, a in zip(np.asarray(centers), np.asarray(widths), np.asarray(amps)):
        r = np.sqrt(np.sum((points - np.asarray(c)) ** 2, axis=-1))
        out = out + a * radial_potential(d, r, float(w), int(p))
    return out
