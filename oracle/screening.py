"""Boundary values by the screening charge (James-type methods) -- oracle.

TEST INFRASTRUCTURE ONLY: used by the tests; never by the product path.

The paper builds on the family of methods that add a harmonic correction to a
homogeneous-Dirichlet solution (Section 1, James 1977 and successors) and
evaluates the harmonic part's boundary values by a volume sum of G against rho
(Section 4), which it prefers because the support of rho stays away from the
boundary and no singular integral appears (Section 2).  This module computes
the same boundary values the James way, for comparison:

* phi* (Section 3) vanishes on the boundary and solves Delta phi* = rho inside.
  Extended by zero outside the box, its Laplacian is rho plus a single layer on
  the boundary whose density is the jump of the normal derivative, -d phi*/dn
  (n the outward normal).  Hence G * rho = phi*_ext + G * (d phi*/dn on the
  boundary), and on the boundary, where phi*_ext = 0,

      g(x) = integral over the boundary of G(|x - s|) sigma(s) dS(s),
      sigma = d phi*/dn                                  (the screening charge).

* sigma comes spectrally from the sine coefficients alpha_k of phi*:
      face x_a = lo (normal -e_a): sigma = -sum_k alpha_k (pi k_a / L_a) prod_{b != a} sin
      face x_a = hi (normal +e_a): sigma =  sum_k alpha_k (pi k_a / L_a) (-1)^{k_a} prod_{b != a} sin
  i.e. face sine coefficients summed over k_a, then a sine synthesis over the
  face's own axes; sigma vanishes on the face's edges.

* The surface integral, face by face, with the trapezoidal rule in each in-face
  direction carrying fourth-order Gregory end weights (3/8, 7/6, 23/24 from
  each edge), the target node itself left out of the sum, and for a target
  inside the face a correction for the singularity of G there:
      3D, G = -1/(4 pi r):   - C(h_b, h_c) sigma(x) / (4 pi)
      2D, G = log(r)/(2 pi):  h log(h / (2 pi)) sigma(x) / (2 pi)
  C(h_b, h_c) is the regularised value of  integral(1/|x|) - h_b h_c sum'(1/|x_j|)
  over the lattice (m h_b, n h_c) (its square-lattice value is
  -4 zeta(1/2) beta(1/2) h), evaluated here by an Ewald split; h log(h / 2 pi)
  is the one-dimensional analogue for log|x|.  Both make the punctured
  trapezoidal rule third-order accurate at the singular point.
  1D: the boundary is two points and the sum is exact.

Unlike the volume sum, this reading is not exact for the discrete problem:
its accuracy is set by the surface quadrature (edges and the singular point),
while phi*'s sine coefficients are spectrally accurate.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc

from . import poisson as P

GREGORY = (3.0 / 8.0, 7.0 / 6.0, 23.0 / 24.0)


def lattice_constant(hb: float, hc: float) -> float:
    """C(h_b, h_c) = integral over R^2 of 1/|x|  -  h_b h_c sum over x_j != 0 of 1/|x_j|
    (regularised; x_j = (m h_b, n h_c)), by the Ewald split
    1/r = erfc(alpha r)/r + erf(alpha r)/r: the first part summed in real space,
    the second through Poisson summation in the reciprocal lattice."""
    a, b = float(hb), float(hc)
    area = a * b
    alpha = 1.5 / np.sqrt(area)
    reach = 12.0
    mr = int(np.ceil(reach / (alpha * a)))
    nr = int(np.ceil(reach / (alpha * b)))
    m, n = np.meshgrid(np.arange(-mr, mr + 1), np.arange(-nr, nr + 1), indexing="ij")
    r = np.hypot(m * a, n * b)
    r[mr, nr] = np.inf
    real = np.sum(erfc(alpha * r) / r)
    km = int(np.ceil(alpha * reach * a / np.pi))
    kn = int(np.ceil(alpha * reach * b / np.pi))
    p, q = np.meshgrid(np.arange(-km, km + 1), np.arange(-kn, kn + 1), indexing="ij")
    k = np.hypot(2 * np.pi * p / a, 2 * np.pi * q / b)
    k[km, kn] = np.inf
    recip = np.sum(2 * np.pi / k * erfc(k / (2 * alpha)))
    return 2 * np.sqrt(np.pi) / alpha - area * real - recip + 2 * alpha * area / np.sqrt(np.pi)


def gregory_weights(M: int) -> np.ndarray:
    """Trapezoid weights on nodes 0..M with fourth-order Gregory end corrections."""
    if M < 6:
        raise ValueError("the end corrections need M >= 6 panels")
    w = np.ones(M + 1)
    for i, v in enumerate(GREGORY):
        w[i] = v
        w[M - i] = v
    return w


def sine_coefficients(rho: np.ndarray, h) -> np.ndarray:
    """alpha_k of phi* (Section 3): beta = prod(2/L) h DST(rho_I), alpha = -beta / (pi^2 sum k^2/L^2)."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    M = np.array(rho.shape) - 1
    L = M * h
    inner = rho[(slice(1, -1),) * d]
    beta = P.dst(inner)
    for ax in range(d):
        beta = beta * (2.0 / L[ax]) * h[ax]
    ks = P._mode_grids(inner.shape)
    q = sum((np.pi * ks[ax] / L[ax]) ** 2 for ax in range(d))
    return -beta / q


def screening_charge(rho: np.ndarray, h):
    """sigma = d phi*/dn on every face: {(axis, side): array over the face nodes}
    (side 0 = low face, 1 = high face; the face array spans all nodes of the
    other axes, edges included, where sigma = 0).  1D: scalars."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    M = np.array(rho.shape) - 1
    L = M * h
    alpha = sine_coefficients(rho, h)
    out = {}
    for a in range(d):
        ka = np.arange(1, M[a], dtype=np.float64)
        wa = np.pi * ka / L[a]
        sh = [1] * d
        sh[a] = M[a] - 1
        lo = -np.sum(alpha * wa.reshape(sh), axis=a)
        hi = np.sum(alpha * (wa * (-1.0) ** ka).reshape(sh), axis=a)
        others = [b for b in range(d) if b != a]
        for side, coef in ((0, lo), (1, hi)):
            if d == 1:
                out[(a, side)] = float(coef)
                continue
            face = np.zeros([M[b] + 1 for b in others])
            face[(slice(1, -1),) * (d - 1)] = P.dst(coef)
            out[(a, side)] = face
    return out


def _face_nodes(n, h, a, side):
    """Coordinates (origin at node 0) of the nodes of face (a, side), in the
    index order of the face arrays."""
    d = len(n)
    others = [b for b in range(d) if b != a]
    grids = np.meshgrid(*[np.arange(n[b]) for b in others], indexing="ij")
    pts = np.zeros(grids[0].shape + (d,))
    pts[..., a] = 0.0 if side == 0 else (n[a] - 1) * h[a]
    for g, b in zip(grids, others):
        pts[..., b] = g * h[b]
    return pts


def screening_boundary_values(rho: np.ndarray, h) -> np.ndarray:
    """Full-grid array holding g on every boundary node (0 inside), from the
    screening charge and the corrected surface trapezoidal rule (module
    docstring).  Every boundary node gets one value: edges and corners sum the
    contributions of all faces like any other target."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    n = rho.shape
    M = [v - 1 for v in n]
    sig = screening_charge(rho, h)
    mask = P.boundary_mask(n)
    targets = np.argwhere(mask)
    xt = targets * h
    g = np.zeros(len(targets))
    if d == 1:
        ends = (0.0, M[0] * h[0])
        for side in (0, 1):
            g += P.green(1, np.abs(xt[:, 0] - ends[side])) * sig[(0, side)]
        out = np.zeros_like(rho)
        out[mask] = g
        return out
    for a in range(d):
        others = [b for b in range(d) if b != a]
        # surface weights: tensor product of Gregory-corrected trapezoid weights
        W = np.ones([M[b] + 1 for b in others])
        for j, b in enumerate(others):
            sh = [1] * (d - 1)
            sh[j] = M[b] + 1
            W = W * (h[b] * gregory_weights(M[b])).reshape(sh)
        if d == 3:
            tau = -lattice_constant(h[others[0]], h[others[1]]) / (4 * np.pi)
        else:
            hb = h[others[0]]
            tau = hb * np.log(hb / (2 * np.pi)) / (2 * np.pi)
        for side in (0, 1):
            s = sig[(a, side)]
            src = _face_nodes(n, h, a, side).reshape(-1, d)
            ws = (W * s).reshape(-1)
            keep = ws != 0.0
            src, ws = src[keep], ws[keep]
            for c0 in range(0, len(targets), 2048):
                t = xt[c0:c0 + 2048]
                r = np.sqrt(((t[:, None, :] - src[None, :, :]) ** 2).sum(-1))
                with np.errstate(divide="ignore"):
                    kern = P.green(d, r)
                kern[r == 0.0] = 0.0  # the target itself is left out of the sum
                g[c0:c0 + 2048] += kern @ ws
            # singular correction for targets on this face (sigma = 0 on its edges)
            on = targets[:, a] == (0 if side == 0 else M[a])
            idx = tuple(targets[on][:, b] for b in others)
            g[on] += tau * s[idx]
    out = np.zeros_like(rho)
    out[mask] = g
    return out


def solve_screening(rho: np.ndarray, h, order: int = 6) -> np.ndarray:
    """phi = phi* + phi_H with phi_H's boundary values from the screening charge
    (the harmonic part as in Section 5)."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    g = screening_boundary_values(rho, h)
    ps = P.phi_star(rho, h)
    if d == 1:
        return ps + P.harmonic_1d(g, h)
    return ps + P.harmonic(g, h, order)
