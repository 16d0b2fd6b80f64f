"""Plain FP64 oracle of the infinite-domain Poisson method (arXiv 2108.11871).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product path.

Everything here follows the paper's steps in its order and notation, with
no blocking, fusion or reordering:

* Section 2: phi = phi_star + phi_H (eqs. PhiStarEqn, PhiHeqn).
* Section 3: phi_star from the discrete sine transform of the interior
  samples of rho, divided by the continuous eigenvalues (eq. for alpha).
* Section 4: boundary values by the trapezoidal sum of G against rho over
  the interior nodes (eq. TrapOrig2D and its 1D/3D analogues), evaluated
  directly (``boundary_values``); the slice-convolution form of the same
  sum (eqs. Trap2D, convolution) is ``boundary_values_fft``.
* Section 5: the compact fourth-order operator L_h (eqs. harmonic4thOrder2D,
  harmonic4thOrder3D), the homogeneous-boundary transfer g~ (eq.
  harmonic4thOrderNH2D), its sine-transform solve, and the sixth-order
  deferred correction (eqs. 6thOrderRelation2D, 6thOrderRelation3D) with
  cubic extrapolation of the right-hand side next to the boundary.
* 1D: exact linear harmonic part (Section 5, first paragraph).

Readings where the paper is silent or garbled (all shared with the GPU path
by specification, never by code):

* grid nodes x_i = a_i + i h_i, i = 0..M_i (the printed node formula mixes up
  the interval end points);
* the 2D compact operator is Delta_h + (h_x^2 + h_y^2)/12 D2_x D2_y, i.e. the
  two printed D2_x D2_y terms carry h_x^2/12 and h_y^2/12 respectively;
  in 3D pair (i, j) carries (h_i^2 + h_j^2)/12;
* the sixth-order right-hand side is the printed sum (with "+" between the
  3D rows), the solution u2 satisfies u2 = g on the boundary;
* the cubic extrapolation fills every interior node with an index equal to
  1 or M_i - 1 from the four nearest core values along that axis
  (weights 4, -6, 4, -1), axis 0 first, then axis 1, then axis 2, each over
  the span already filled; core = all indices in [2, M_i - 2];
* every boundary node (faces, edges, corners) gets g;
* rho on boundary nodes is ignored;
* the 2D Green's function carries its 1/(2 pi) factor.

Arrays: grids are numpy arrays of shape n = (n_0, ..., n_{d-1}); node
(i_0, ..., i_{d-1}) sits at x = a + i h.  ``interior`` arrays have shape
(n_0 - 2, ..., n_{d-1} - 2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_QUAD_SRC = os.path.join(_HERE, "quad.c")
_QUAD_LIB = os.path.join(_HERE, "liboracle_quad.so")
_quad_lock = threading.Lock()
_quad = None


def build_quad(force: bool = False) -> str:
    """Compile the direct-quadrature helper (plain C, OpenMP, no fast-math)."""
    if force or not os.path.exists(_QUAD_LIB) or (
        os.path.getmtime(_QUAD_LIB) < os.path.getmtime(_QUAD_SRC)
    ):
        tmp = _QUAD_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _QUAD_SRC, "-lm"]
        )
        os.replace(tmp, _QUAD_LIB)
    return _QUAD_LIB


def _quad_lib():
    global _quad
    with _quad_lock:
        if _quad is None:
            lib = ctypes.CDLL(build_quad())
            lib.oracle_boundary_direct.restype = ctypes.c_int
            lib.oracle_boundary_direct.argtypes = [
                ctypes.c_int,
                ctypes.POINTER(ctypes.c_int64),
                ctypes.POINTER(ctypes.c_double),
                ctypes.POINTER(ctypes.c_double),
                ctypes.c_int64,
                ctypes.POINTER(ctypes.c_int64),
                ctypes.POINTER(ctypes.c_double),
            ]
            lib.oracle_boundary_adjoint.restype = ctypes.c_int
            lib.oracle_boundary_adjoint.argtypes = [
                ctypes.c_int,
                ctypes.POINTER(ctypes.c_int64),
                ctypes.POINTER(ctypes.c_double),
                ctypes.c_int64,
                ctypes.POINTER(ctypes.c_int64),
                ctypes.POINTER(ctypes.c_double),
                ctypes.POINTER(ctypes.c_double),
            ]
            _quad = lib
    return _quad


# ----------------------------------------------------------------------------
# Green's function (Section 1)
# ----------------------------------------------------------------------------
def green(d: int, r):
    """Free-space Green's function of the Laplacian: r/2, log(r)/(2 pi), -1/(4 pi r)."""
    r = np.asarray(r, dtype=np.float64)
    if d == 1:
        return 0.5 * r
    if d == 2:
        return np.log(r) / (2.0 * np.pi)
    if d == 3:
        return -1.0 / (4.0 * np.pi * r)
    raise ValueError("d must be 1, 2 or 3")


# ----------------------------------------------------------------------------
# Discrete sine transform (Section 3), dense O(n^2) matrices
# ----------------------------------------------------------------------------
def sine_matrix(M: int) -> np.ndarray:
    """S[k-1, j-1] = sin(pi k j / M) for k, j = 1..M-1.

    The integer k*j is reduced modulo 2M before scaling so that the argument
    of sin never exceeds 2 pi (keeps every entry accurate to a few ulps).
    """
    k = np.arange(1, M, dtype=np.int64)
    r = np.outer(k, k) % (2 * M)
    return np.sin(np.pi * r.astype(np.float64) / M)


def _apply_along(mat: np.ndarray, f: np.ndarray, axis: int) -> np.ndarray:
    out = np.tensordot(mat, f, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def dst(f: np.ndarray) -> np.ndarray:
    """Raw multi-dimensional DST-I of an interior array: sum_j f_j prod sin(pi k j / M)."""
    out = f
    for ax in range(f.ndim):
        out = _apply_along(sine_matrix(f.shape[ax] + 1), out, ax)
    return out


def _mode_grids(shape_interior):
    """k_i = 1..M_i-1 along each axis, broadcastable."""
    d = len(shape_interior)
    ks = []
    for ax, m in enumerate(shape_interior):
        k = np.arange(1, m + 1, dtype=np.float64)
        sh = [1] * d
        sh[ax] = m
        ks.append(k.reshape(sh))
    return ks


# ----------------------------------------------------------------------------
# phi_star (Section 3)
# ----------------------------------------------------------------------------
def phi_star(rho: np.ndarray, h) -> np.ndarray:
    """Sine-series solution of Delta phi* = rho with phi* = 0 on the boundary.

    beta_k = prod(2/L_i) sum_j rho_j prod sin(k_i pi (x_i - a_i)/L_i) prod h_i
    alpha_k = -beta_k / (pi^2 sum_i k_i^2 / L_i^2)
    phi*_j = sum_k alpha_k prod sin(...)
    """
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(h, dtype=np.float64)
    M = np.array(rho.shape) - 1
    L = M * h
    inner = rho[(slice(1, -1),) * d]
    beta = dst(inner)
    for ax in range(d):
        beta = beta * (2.0 / L[ax]) * h[ax]
    ks = _mode_grids(inner.shape)
    denom = sum((np.pi * ks[ax] / L[ax]) ** 2 for ax in range(d))
    alpha = -beta / denom
    out = np.zeros_like(rho)
    out[(slice(1, -1),) * d] = dst(alpha)
    return out


# ----------------------------------------------------------------------------
# Boundary values (Section 4)
# ----------------------------------------------------------------------------
def boundary_mask(n) -> np.ndarray:
    n = tuple(int(v) for v in n)
    mask = np.zeros(n, dtype=bool)
    for ax in range(len(n)):
        idx = [slice(None)] * len(n)
        idx[ax] = 0
        mask[tuple(idx)] = True
        idx[ax] = -1
        mask[tuple(idx)] = True
    return mask


def boundary_values_at(rho: np.ndarray, h, targets: np.ndarray) -> np.ndarray:
    """Trapezoidal sum prod(h) sum_{s interior} G(|x_t - x_s|) rho_s at listed nodes.

    ``targets`` is an (ntargets, d) integer array of node indices.
    """
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    d = rho.ndim
    n = np.ascontiguousarray(rho.shape, dtype=np.int64)
    hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    t = np.ascontiguousarray(targets, dtype=np.int64).reshape(-1, d)
    out = np.zeros(t.shape[0], dtype=np.float64)
    lib = _quad_lib()
    rc = lib.oracle_boundary_direct(
        d,
        n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        hh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        t.shape[0],
        t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
    )
    if rc != 0:
        raise RuntimeError("oracle_boundary_direct failed (%d)" % rc)
    return out


def boundary_values(rho: np.ndarray, h) -> np.ndarray:
    """Full-grid array holding g on every boundary node (0 inside), direct sums."""
    rho = np.asarray(rho, dtype=np.float64)
    mask = boundary_mask(rho.shape)
    targets = np.argwhere(mask)
    g = np.zeros_like(rho)
    g[mask] = boundary_values_at(rho, h, targets)
    return g


def boundary_values_fft(rho: np.ndarray, h) -> np.ndarray:
    """Same sums as ``boundary_values`` via the slice-convolution form (Section 4).

    For each axis a and each interior slice p perpendicular to it, the values
    on the two faces a = 0 and a = M_a are discrete convolutions over the
    remaining axes of rho(slice p) with G(sqrt((p h_a)^2 + |delta|^2)) and
    G(sqrt(((M_a - p) h_a)^2 + |delta|^2)); the convolutions are summed over p.
    Each convolution is evaluated exactly by a zero-padded FFT of length 2 M
    per axis (any length >= 2M - 1 reproduces the direct sum).
    Edges and corners take the value from the lowest axis whose face holds them.
    """
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    n = rho.shape
    M = [v - 1 for v in n]
    vol = float(np.prod(h))
    g = np.zeros_like(rho)
    written = np.zeros(n, dtype=bool)
    if d == 1:
        return boundary_values(rho, h)
    inner = rho[(slice(1, -1),) * d]
    for a in range(d):
        others = [b for b in range(d) if b != a]
        P = [2 * M[b] for b in others]
        # offsets delta_b in [-M_b+1, M_b] laid out circularly
        offs = []
        for b, Pb in zip(others, P):
            o = np.arange(Pb)
            o = np.where(o <= M[b], o, o - Pb)
            offs.append(o.astype(np.float64) * h[b])
        mesh = np.meshgrid(*offs, indexing="ij")
        r2_in = sum(m * m for m in mesh)
        acc = [np.zeros([M[b] + 1 for b in others]), np.zeros([M[b] + 1 for b in others])]
        for p in range(1, M[a]):
            sl = np.take(inner, p - 1, axis=a)
            pad = np.zeros(P)
            pad[tuple(slice(1, M[b]) for b in others)] = sl
            fs = np.fft.fftn(pad)
            for face, dist in ((0, p * h[a]), (1, (M[a] - p) * h[a])):
                K = green(d, np.sqrt(dist * dist + r2_in))
                conv = np.fft.ifftn(fs * np.fft.fftn(K)).real
                acc[face] += conv[tuple(slice(0, M[b] + 1) for b in others)]
        for face in (0, 1):
            idx = [slice(None)] * d
            idx[a] = 0 if face == 0 else M[a]
            idx = tuple(idx)
            sel = ~written[idx]
            vals = acc[face] * vol
            gv = g[idx]
            gv[sel] = vals[sel]
            g[idx] = gv
            w = written[idx]
            w[:] = True
            written[idx] = w
    return g


# ----------------------------------------------------------------------------
# Difference operators (Section 5)
# ----------------------------------------------------------------------------
def d2(u: np.ndarray, axis: int, hax: float) -> np.ndarray:
    """Three-point second difference [1, -2, 1]/h^2 along ``axis``; that axis shrinks by 2."""
    n = u.shape[axis]

    def sl(a, b):
        s = [slice(None)] * u.ndim
        s[axis] = slice(a, b)
        return tuple(s)

    return (u[sl(2, n)] - 2.0 * u[sl(1, n - 1)] + u[sl(0, n - 2)]) / (hax * hax)


def _restrict(v: np.ndarray, shrink) -> np.ndarray:
    """Cut an array by ``shrink[ax]`` nodes at each end of every axis."""
    idx = tuple(slice(s, v.shape[ax] - s) for ax, s in enumerate(shrink))
    return v[idx]


def compact_coeff(h, i: int, j: int) -> float:
    """Coefficient of D2_i D2_j in the compact fourth-order operator: (h_i^2 + h_j^2)/12."""
    return (h[i] ** 2 + h[j] ** 2) / 12.0


def apply_Lh(u: np.ndarray, h) -> np.ndarray:
    """L_h u = sum_i D2_i u + sum_{i<j} (h_i^2 + h_j^2)/12 D2_i D2_j u at interior nodes."""
    d = u.ndim
    out = 0.0
    for i in range(d):
        v = d2(u, i, h[i])
        out = out + _restrict(v, [0 if ax == i else 1 for ax in range(d)])
    for i in range(d):
        for j in range(i + 1, d):
            v = d2(d2(u, j, h[j]), i, h[i])
            out = out + compact_coeff(h, i, j) * _restrict(
                v, [0 if ax in (i, j) else 1 for ax in range(d)]
            )
    return out


def transfer(g_full: np.ndarray, h) -> np.ndarray:
    """g~ = -(L_h B) on interior nodes, B = g on the boundary and 0 inside (eq. harmonic4thOrderNH2D)."""
    B = np.array(g_full, dtype=np.float64)
    B[(slice(1, -1),) * B.ndim] = 0.0
    return -apply_Lh(B, h)


def eigen_L0(shape_interior, h) -> np.ndarray:
    """Eigenvalues of L_0 on the discrete sine modes:
    Lambda(k) = sum_i lam_i + sum_{i<j} (h_i^2 + h_j^2)/12 lam_i lam_j,
    lam_i = -(4/h_i^2) sin^2(pi k_i / (2 M_i))."""
    d = len(shape_interior)
    ks = _mode_grids(shape_interior)
    lam = []
    for ax in range(d):
        M = shape_interior[ax] + 1
        lam.append(-(4.0 / h[ax] ** 2) * np.sin(np.pi * ks[ax] / (2.0 * M)) ** 2)
    out = sum(lam)
    for i in range(d):
        for j in range(i + 1, d):
            out = out + compact_coeff(h, i, j) * lam[i] * lam[j]
    return out


def solve_L0(f: np.ndarray, h) -> np.ndarray:
    """Solve L_0 u = f on the interior (homogeneous Dirichlet) by sine transforms."""
    f = np.asarray(f, dtype=np.float64)
    c = dst(f)
    for ax in range(f.ndim):
        c = c * (2.0 / (f.shape[ax] + 1))
    c = c / eigen_L0(f.shape, h)
    return dst(c)


def rhs6_core(u_full: np.ndarray, h) -> np.ndarray:
    """Sixth-order right-hand side on the core (all indices in [2, M_i - 2]).

    Sum over pairs i < j of
      (h_i^4/240 + h_i^2 h_j^2/144) D2_i D2_i D2_j u
    + (h_j^4/240 + h_i^2 h_j^2/144) D2_j D2_i D2_j u     (eqs. 6thOrderRelation2D/3D)
    """
    d = u_full.ndim
    out = 0.0
    for i in range(d):
        for j in range(i + 1, d):
            cij = h[i] ** 4 / 240.0 + h[i] ** 2 * h[j] ** 2 / 144.0
            cji = h[j] ** 4 / 240.0 + h[i] ** 2 * h[j] ** 2 / 144.0
            dij = d2(u_full, j, h[j])  # shrinks j by 1 each side
            t1 = d2(d2(dij, i, h[i]), i, h[i])  # i shrinks by 2 each side
            t2 = d2(d2(dij, j, h[j]), i, h[i])  # j by 2, i by 1
            t1 = _restrict(t1, [0 if ax == i else (1 if ax == j else 2) for ax in range(d)])
            t2 = _restrict(t2, [0 if ax == j else (1 if ax == i else 2) for ax in range(d)])
            out = out + cij * t1 + cji * t2
    return out


def extrapolate(core: np.ndarray) -> np.ndarray:
    """Cubic extrapolation of the right-hand side to the nodes next to the boundary.

    ``core`` holds the values at indices 2..M_i-2; the result covers 1..M_i-1.
    Index 1 gets 4 R[2] - 6 R[3] + 4 R[4] - R[5] (and symmetrically at
    M_i - 1), axis 0 first, each axis over the span filled so far.
    """
    d = core.ndim
    R = np.zeros([s + 2 for s in core.shape])
    R[(slice(1, -1),) * d] = core
    filled = [False] * d
    for ax in range(d):
        span = []
        for b in range(d):
            if b == ax:
                span.append(None)
            else:
                span.append(slice(None) if filled[b] else slice(1, R.shape[b] - 1))

        def at(pos):
            return tuple(pos if b == ax else span[b] for b in range(d))

        m = R.shape[ax]
        R[at(0)] = 4 * R[at(1)] - 6 * R[at(2)] + 4 * R[at(3)] - R[at(4)]
        R[at(m - 1)] = 4 * R[at(m - 2)] - 6 * R[at(m - 3)] + 4 * R[at(m - 4)] - R[at(m - 5)]
        filled[ax] = True
    return R


def rhs6(u_full: np.ndarray, h) -> np.ndarray:
    """Sixth-order right-hand side on all interior nodes (core values + extrapolation)."""
    return extrapolate(rhs6_core(u_full, h))


# ----------------------------------------------------------------------------
# Harmonic correction (Section 5) and the full method (Section 2)
# ----------------------------------------------------------------------------
def harmonic(g_full: np.ndarray, h, order: int) -> np.ndarray:
    """Discrete harmonic function with boundary values g: 4th or 6th order."""
    g_full = np.asarray(g_full, dtype=np.float64)
    d = g_full.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    inner = (slice(1, -1),) * d
    gt = transfer(g_full, h)
    u1 = np.array(g_full)
    u1[inner] = solve_L0(gt, h)
    if order == 4:
        return u1
    if order != 6:
        raise ValueError("order must be 4 or 6")
    R = rhs6(u1, h)
    u2 = np.array(g_full)
    u2[inner] = solve_L0(gt + R, h)
    return u2


def harmonic_1d(g_full: np.ndarray, h) -> np.ndarray:
    """Exact 1D harmonic part: the linear function through the two end values."""
    n = g_full.shape[0]
    t = np.arange(n, dtype=np.float64) / (n - 1)
    return g_full[0] + (g_full[-1] - g_full[0]) * t


def solve(rho: np.ndarray, h, order: int = 6, boundary: str = "direct") -> np.ndarray:
    """phi = phi_star + phi_H at every node (interior), phi = g on the boundary."""
    rho = np.asarray(rho, dtype=np.float64)
    d = rho.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    ps = phi_star(rho, h)
    g = boundary_values(rho, h) if boundary == "direct" else boundary_values_fft(rho, h)
    if d == 1:
        return ps + harmonic_1d(g, h)
    return ps + harmonic(g, h, order)


# ----------------------------------------------------------------------------
# Adjoint of the whole map rho -> phi (for gradients)
# ----------------------------------------------------------------------------
# phi = A rho is linear in rho (the boundary entries of rho are ignored).
# Each forward step above is linear; its transpose is written out below and
# chained in reverse order.  Pinned by <A v, w> = <v, A^T w> and by dense
# matrices of A on tiny grids.


def boundary_values_T(lam_full: np.ndarray, h) -> np.ndarray:
    """Transpose of ``boundary_values``: rho_bar(s) = prod(h) sum_b G(|x_b - x_s|) lam(b)
    over the boundary nodes b, for every interior node s (0 on the boundary)."""
    lam_full = np.asarray(lam_full, dtype=np.float64)
    d = lam_full.ndim
    n = np.ascontiguousarray(lam_full.shape, dtype=np.int64)
    hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    mask = boundary_mask(lam_full.shape)
    t = np.ascontiguousarray(np.argwhere(mask), dtype=np.int64)
    lam = np.ascontiguousarray(lam_full[mask])
    out = np.zeros(lam_full.shape)
    lib = _quad_lib()
    rc = lib.oracle_boundary_adjoint(
        d,
        n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        hh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        t.shape[0],
        t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
    )
    if rc != 0:
        raise RuntimeError("oracle_boundary_adjoint failed (%d)" % rc)
    return out


def d2_T(v: np.ndarray, axis: int, hax: float) -> np.ndarray:
    """Transpose of ``d2``: the input's ``axis`` grows by 2."""
    shape = list(v.shape)
    shape[axis] += 2
    out = np.zeros(shape)
    n = shape[axis]

    def sl(a, b):
        s = [slice(None)] * v.ndim
        s[axis] = slice(a, b)
        return tuple(s)

    w = v / (hax * hax)
    out[sl(2, n)] += w
    out[sl(1, n - 1)] -= 2.0 * w
    out[sl(0, n - 2)] += w
    return out


def _restrict_T(v: np.ndarray, shrink) -> np.ndarray:
    """Transpose of ``_restrict``: zero padding."""
    return np.pad(v, [(s, s) for s in shrink])


def apply_Lh_T(y: np.ndarray, h) -> np.ndarray:
    """Transpose of ``apply_Lh`` (interior values -> full grid)."""
    d = y.ndim
    out = 0.0
    for i in range(d):
        out = out + d2_T(_restrict_T(y, [0 if ax == i else 1 for ax in range(d)]), i, h[i])
    for i in range(d):
        for j in range(i + 1, d):
            v = _restrict_T(y, [0 if ax in (i, j) else 1 for ax in range(d)])
            out = out + compact_coeff(h, i, j) * d2_T(d2_T(v, i, h[i]), j, h[j])
    return out


def transfer_T(y: np.ndarray, h) -> np.ndarray:
    """Transpose of ``transfer``: interior values -> boundary nodes (0 inside)."""
    out = -apply_Lh_T(y, h)
    out[(slice(1, -1),) * y.ndim] = 0.0
    return out


def rhs6_core_T(core_bar: np.ndarray, h) -> np.ndarray:
    """Transpose of ``rhs6_core`` (core values -> full grid)."""
    d = core_bar.ndim
    out = 0.0
    for i in range(d):
        for j in range(i + 1, d):
            cij = h[i] ** 4 / 240.0 + h[i] ** 2 * h[j] ** 2 / 144.0
            cji = h[j] ** 4 / 240.0 + h[i] ** 2 * h[j] ** 2 / 144.0
            t1 = _restrict_T(cij * core_bar, [0 if ax == i else (1 if ax == j else 2) for ax in range(d)])
            t2 = _restrict_T(cji * core_bar, [0 if ax == j else (1 if ax == i else 2) for ax in range(d)])
            v1 = d2_T(d2_T(t1, i, h[i]), i, h[i])
            v2 = d2_T(d2_T(t2, i, h[i]), j, h[j])
            out = out + d2_T(v1 + v2, j, h[j])
    return out


def extrapolate_T(Rbar: np.ndarray) -> np.ndarray:
    """Transpose of ``extrapolate`` (interior-size array -> core-size array)."""
    R = np.array(Rbar, dtype=np.float64)
    d = R.ndim
    filled = [True] * d
    for ax in reversed(range(d)):
        filled[ax] = False
        span = []
        for b in range(d):
            if b == ax:
                span.append(None)
            else:
                span.append(slice(None) if filled[b] else slice(1, R.shape[b] - 1))

        def at(pos):
            return tuple(pos if b == ax else span[b] for b in range(d))

        m = R.shape[ax]
        lo = R[at(0)].copy()
        hi = R[at(m - 1)].copy()
        R[at(0)] = 0.0
        R[at(m - 1)] = 0.0
        for k, w in zip((1, 2, 3, 4), (4.0, -6.0, 4.0, -1.0)):
            R[at(k)] += w * lo
            R[at(m - 1 - k)] += w * hi
    return R[(slice(1, -1),) * d]


def adjoint(w: np.ndarray, h, order: int = 6) -> np.ndarray:
    """rho_bar = A^T w for the map rho -> phi computed by ``solve`` (boundary of rho_bar = 0)."""
    w = np.asarray(w, dtype=np.float64)
    d = w.ndim
    h = np.asarray(np.broadcast_to(np.asarray(h, np.float64), (d,)))
    inner = (slice(1, -1),) * d
    mask = boundary_mask(w.shape)
    lam = np.where(mask, w, 0.0)  # w on the boundary: phi = g there
    if d == 1:
        M = w.shape[0] - 1
        t = np.arange(1, M, dtype=np.float64) / M
        lam[0] += np.sum(w[1:-1] * (1.0 - t))
        lam[-1] += np.sum(w[1:-1] * t)
    else:
        wI = w[inner]
        a = solve_L0(wI, h)  # L_0^-1 is symmetric
        gt_bar = a
        if order == 6:
            core_bar = extrapolate_T(a)
            u1_bar = rhs6_core_T(core_bar, h)
            lam = lam + np.where(mask, u1_bar, 0.0)  # R_boundary^T a
            b = solve_L0(u1_bar[inner], h)  # L_0^-1 R_interior^T a
            gt_bar = a + b
        elif order != 4:
            raise ValueError("order must be 4 or 6")
        lam = lam + transfer_T(gt_bar, h)
    out = phi_star(w, h)  # phi_star's map is symmetric on the interior
    out = out + boundary_values_T(lam, h)
    out[mask] = 0.0
    return out
