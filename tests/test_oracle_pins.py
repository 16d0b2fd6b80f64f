"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
solutions, exact identities, brute force written independently, dense linear
algebra assembled from the printed stencils, or measured convergence orders.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import poisson as P
from paper_2108_11871_amd import inputs as I


def _grid(n, lo, hi):
    n = np.asarray(n)
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    h = (hi - lo) / (n - 1)
    xs = [lo[a] + h[a] * np.arange(n[a]) for a in range(len(n))]
    return h, np.meshgrid(*xs, indexing="ij")


# ---------------------------------------------------------------------------
# Section 3: sine transforms and phi_star
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("M", [2, 3, 8, 37, 64])
def test_sine_matrix_squares_to_half_M(M):
    S = P.sine_matrix(M)
    assert np.allclose(S @ S, (M / 2.0) * np.eye(M - 1), atol=1e-13 * M)


def test_sine_matrix_matches_definition_small():
    M = 5
    S = P.sine_matrix(M)
    for k in range(1, M):
        for j in range(1, M):
            assert abs(S[k - 1, j - 1] - math.sin(math.pi * k * j / M)) < 1e-15


@pytest.mark.parametrize("d", [1, 2, 3])
def test_phi_star_of_a_sine_mode_is_exact(d):
    # rho = prod sin(k_i pi (x_i - a_i)/L_i) has phi* = -rho / (pi^2 sum k_i^2/L_i^2)
    n = [9, 12, 7][:d]
    lo = [-1.0, -0.3, 0.2][:d]
    hi = [1.0, 1.4, 0.9][:d]
    ks = [3, 2, 5][:d]
    h, X = _grid(n, lo, hi)
    L = np.asarray(hi) - np.asarray(lo)
    rho = np.ones(X[0].shape)
    for a in range(d):
        rho = rho * np.sin(ks[a] * np.pi * (X[a] - lo[a]) / L[a])
    expect = -rho / sum((np.pi * ks[a] / L[a]) ** 2 for a in range(d))
    inner = (slice(1, -1),) * d
    got = P.phi_star(rho, h)
    assert np.abs(got[inner] - expect[inner]).max() < 1e-14 * np.abs(expect).max()
    assert np.all(P.boundary_mask(rho.shape) <= (got == 0.0))


# ---------------------------------------------------------------------------
# Section 4: boundary values
# ---------------------------------------------------------------------------
def _brute_force_boundary(rho, h):
    """Independent pure-Python quadrature: loops over (target, source) pairs."""
    d = rho.ndim
    n = rho.shape
    out = {}
    vol = float(np.prod(h))
    src = [idx for idx in np.ndindex(*n) if all(0 < idx[a] < n[a] - 1 for a in range(d))]
    for t in np.ndindex(*n):
        if all(0 < t[a] < n[a] - 1 for a in range(d)):
            continue
        acc = 0.0
        for s in src:
            r = math.sqrt(sum(((t[a] - s[a]) * h[a]) ** 2 for a in range(d)))
            if d == 1:
                G = r / 2.0
            elif d == 2:
                G = math.log(r) / (2.0 * math.pi)
            else:
                G = -1.0 / (4.0 * math.pi * r)
            acc += G * rho[s]
        out[t] = acc * vol
    return out


@pytest.mark.parametrize("shape", [(9,), (7, 9), (5, 6, 7)])
def test_boundary_direct_matches_python_brute_force(shape):
    rng = np.random.default_rng(11)
    rho = rng.standard_normal(shape)  # boundary entries must be ignored
    h = np.array([0.3, 0.17, 0.41][: len(shape)])
    g = P.boundary_values(rho, h)
    ref = _brute_force_boundary(rho, h)
    scale = max(abs(v) for v in ref.values())
    for t, v in ref.items():
        assert abs(g[t] - v) <= 1e-13 * scale


def test_boundary_fft_form_matches_direct_sums():
    rho, h, _ = I.workload_bumps((17, 21, 19), seed=5, scale=[1.0, 1.3, 0.9])
    g1 = P.boundary_values(rho, h)
    g2 = P.boundary_values_fft(rho, h)
    m = P.boundary_mask(rho.shape)
    assert np.abs(g1 - g2)[m].max() < 1e-13 * np.abs(g1[m]).max()
    rho2, h2, _ = I.workload_bumps((33, 26), seed=6)
    g1 = P.boundary_values(rho2, h2)
    g2 = P.boundary_values_fft(rho2, h2)
    m = P.boundary_mask(rho2.shape)
    assert np.abs(g1 - g2)[m].max() < 1e-13 * np.abs(g1[m]).max()


@pytest.mark.parametrize("d,n", [(2, 49), (3, 41)])
def test_boundary_values_converge_spectrally_to_closed_form(d, n):
    # Compact bump well inside the box: the trapezoidal sum is spectrally accurate.
    eps, p = 0.45, 12
    c = np.array([0.1, -0.05, 0.07])[:d]
    rho = I.radial_bump((n,) * d, eps, p, center=c)
    h = I.grid_spacing((n,) * d)
    g = P.boundary_values(rho, h)
    _, X = _grid((n,) * d, [-1.0] * d, [1.0] * d)
    r = np.sqrt(sum((X[a] - c[a]) ** 2 for a in range(d)))
    ex = CF.radial_potential(d, r, eps, p)
    m = P.boundary_mask(rho.shape)
    assert np.abs(g - ex)[m].max() < 1e-9 * np.abs(ex[m]).max()


def test_closed_form_2d_satisfies_poisson_and_continuity():
    eps, p = 0.7, 5
    r = np.linspace(0.05, 1.5, 2001)
    f = CF.radial_potential(2, r, eps, p)
    dr = r[1] - r[0]
    lap = (f[2:] - 2 * f[1:-1] + f[:-2]) / dr**2 + (f[2:] - f[:-2]) / (2 * dr) / r[1:-1]
    rho = np.where(r[1:-1] < eps, (1 - r[1:-1] ** 2 / eps**2) ** p, 0.0)
    assert np.abs(lap - rho).max() < 1e-4
    a = CF.radial_potential(2, np.array([eps - 1e-12, eps + 1e-12]), eps, p)
    assert abs(a[0] - a[1]) < 1e-10


def test_closed_form_3d_satisfies_poisson_and_continuity():
    eps, p = 0.6, 6
    r = np.linspace(0.05, 1.5, 2001)
    f = CF.radial_potential(3, r, eps, p)
    dr = r[1] - r[0]
    lap = (f[2:] - 2 * f[1:-1] + f[:-2]) / dr**2 + (f[2:] - f[:-2]) / dr / r[1:-1]
    rho = np.where(r[1:-1] < eps, (1 - r[1:-1] ** 2 / eps**2) ** p, 0.0)
    assert np.abs(lap - rho).max() < 1e-4
    a = CF.radial_potential(3, np.array([eps - 1e-12, eps + 1e-12]), eps, p)
    assert abs(a[0] - a[1]) < 1e-10
    # far field is -Q/(4 pi r) with Q the total charge
    Q = 1.0 / CF.unit_gamma(3, eps, p)
    assert abs(CF.radial_potential(3, np.array([2.0]), eps, p)[0] + Q / (8 * math.pi)) < 1e-15


# ---------------------------------------------------------------------------
# Section 5: difference operators, the compact operator and its DST solve
# ---------------------------------------------------------------------------
def _dense_L0(shape_int, h):
    """Assemble L_0 from the printed stencils ([1,-2,1]/h^2 and the 9-point product)."""
    d = len(shape_int)
    idx = {t: i for i, t in enumerate(np.ndindex(*shape_int))}
    A = np.zeros((len(idx), len(idx)))
    w1 = {-1: 1.0, 0: -2.0, 1: 1.0}
    for t, row in idx.items():

        def add(off, w):
            s = tuple(t[a] + off[a] for a in range(d))
            if s in idx:
                A[row, idx[s]] += w

        for i in range(d):
            for o, w in w1.items():
                off = [0] * d
                off[i] = o
                add(off, w / h[i] ** 2)
        for i in range(d):
            for j in range(i + 1, d):
                c = (h[i] ** 2 + h[j] ** 2) / 12.0
                for oi, wi in w1.items():
                    for oj, wj in w1.items():
                        off = [0] * d
                        off[i] = oi
                        off[j] = oj
                        add(off, c * wi * wj / (h[i] ** 2 * h[j] ** 2))
    return A


@pytest.mark.parametrize("shape_int,h", [((7, 9), (0.2, 0.13)), ((5, 6, 7), (0.3, 0.11, 0.2))])
def test_L0_sine_solve_matches_dense_LU(shape_int, h):
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape_int)
    A = _dense_L0(shape_int, np.asarray(h))
    ref = np.linalg.solve(A, f.ravel()).reshape(shape_int)
    got = P.solve_L0(f, np.asarray(h))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_compact_eigenvalues_negative_for_extreme_aspect_ratios():
    for h in [(1.0, 1e-3, 1e-3), (1e-3, 1.0, 30.0), (0.1, 0.1, 0.1)]:
        lam = P.eigen_L0((6, 7, 8), np.asarray(h))
        assert np.all(lam < 0)


def test_sixth_order_rhs_coefficients_on_polynomials():
    # D2_x^2 D2_y of x^4 y^2 is exactly 48, and D2_x D2_y^2 of it is exactly 0;
    # so R = 48 (h_x^4/240 + h_x^2 h_y^2/144) on the core.  Swapping roles
    # pins which coefficient goes with which term.
    h, (X, Y) = _grid((12, 14), (-1.0, -0.6), (0.9, 1.1))
    R = P.rhs6_core(X**4 * Y**2, h)
    cxy = h[0] ** 4 / 240 + h[0] ** 2 * h[1] ** 2 / 144
    assert np.allclose(R, 48 * cxy, rtol=1e-9, atol=0)
    R = P.rhs6_core(X**2 * Y**4, h)
    cyx = h[1] ** 4 / 240 + h[0] ** 2 * h[1] ** 2 / 144
    assert np.allclose(R, 48 * cyx, rtol=1e-9, atol=0)
    # 3D: x^4 z^2 gives only the (x, z) pair's D2_x^2 D2_z term
    h, (X, Y, Z) = _grid((10, 11, 12), (-1.0, -0.6, -0.7), (0.9, 1.1, 0.8))
    R = P.rhs6_core(X**4 * Z**2, h)
    cxz = h[0] ** 4 / 240 + h[0] ** 2 * h[2] ** 2 / 144
    assert np.allclose(R, 48 * cxz, rtol=1e-9, atol=0)


def test_extrapolation_reproduces_tensor_cubics():
    h, (X, Y, Z) = _grid((11, 12, 13), (-1.0, -1.0, -1.0), (1.0, 1.2, 0.8))
    f = (1 + X - 2 * X**3) * (0.5 - Y**2 + Y**3) * (2 + Z + Z**2 - 0.3 * Z**3)
    core = f[2:-2, 2:-2, 2:-2]
    got = P.extrapolate(core)
    assert np.abs(got - f[1:-1, 1:-1, 1:-1]).max() < 1e-12 * np.abs(f).max()


def _harmonic_polys_2d(X, Y):
    z = X + 1j * Y
    return [np.real(z**k) for k in range(1, 6)] + [np.imag(z**k) for k in range(1, 6)]


def _harmonic_polys_3d(X, Y, Z):
    out = [X**2 - Y**2, X * Y * Z, X**3 - 3 * X * Y**2, X**2 * Z + Y**2 * Z - 2.0 * Z**3 / 3.0]
    out.append(np.real((X + 1j * Y) ** 5))
    out.append(np.real((Y + 1j * Z) ** 4))
    out.append(X * Y * Z * (X**2 - Y**2))
    return out


@pytest.mark.parametrize("order", [4, 6])
def test_harmonic_polynomials_reproduced_to_rounding(order):
    h, (X, Y) = _grid((13, 17), (-1.0, -0.7), (1.2, 0.9))
    for u in _harmonic_polys_2d(X, Y):
        v = P.harmonic(np.where(P.boundary_mask(u.shape), u, 0.0), h, order)
        assert np.abs(v - u).max() < 1e-12 * np.abs(u).max()
    h, (X, Y, Z) = _grid((10, 12, 11), (-1.0, -0.7, -0.9), (1.2, 0.9, 1.1))
    for u in _harmonic_polys_3d(X, Y, Z):
        v = P.harmonic(np.where(P.boundary_mask(u.shape), u, 0.0), h, order)
        assert np.abs(v - u).max() < 1e-12 * np.abs(u).max()


def _rate_3d(order, sizes):
    errs, hs = [], []
    for n in sizes:
        shape = (n, int(n * 1.25), int(n * 0.8))
        h, (X, Y, Z) = _grid(shape, (-1.0, -0.7, -1.2), (1.0, 1.1, 0.9))
        a, b = 0.7, 0.9
        u = np.exp(a * X + b * Y) * np.cos(math.hypot(a, b) * Z)
        v = P.harmonic(np.where(P.boundary_mask(u.shape), u, 0.0), h, order)
        errs.append(np.abs(v - u).max())
        hs.append(h.max())
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def _rate_2d(order, sizes):
    errs, hs = [], []
    for n in sizes:
        h, (X, Y) = _grid((n, int(n * 1.3)), (-1.0, -0.8), (1.0, 1.2))
        u = np.exp(1.3 * X) * np.cos(1.3 * Y)
        v = P.harmonic(np.where(P.boundary_mask(u.shape), u, 0.0), h, order)
        errs.append(np.abs(v - u).max())
        hs.append(h.max())
    return np.polyfit(np.log(hs), np.log(errs), 1)[0]


def test_harmonic_part_is_fourth_and_sixth_order_3d():
    assert 3.8 < _rate_3d(4, (17, 25, 33)) < 4.3
    assert 5.7 < _rate_3d(6, (17, 25, 33)) < 6.4


def test_harmonic_part_is_fourth_and_sixth_order_2d():
    assert 3.8 < _rate_2d(4, (17, 33, 65)) < 4.3
    assert 5.7 < _rate_2d(6, (17, 33, 65)) < 6.4


# ---------------------------------------------------------------------------
# Full method (Section 2)
# ---------------------------------------------------------------------------
def test_full_solve_2d_single_bump_matches_closed_form():
    rho, h, meta = I.workload_2d_single(65)
    phi = P.solve(rho, h, 4)
    _, (X, Y) = _grid((65, 65), (-1.0, -1.0), (1.0, 1.0))
    ex = CF.radial_potential(2, np.sqrt(X**2 + Y**2), meta["eps"], meta["p"])
    assert np.abs(phi - ex).max() < 1e-10 * np.abs(ex).max()


def test_full_solve_3d_bump_sum_converges_to_closed_form():
    errs = []
    for n in (33, 49):
        rho, h, meta = I.workload_bumps_3d(n, seed=1)
        phi = P.solve(rho, h, 6)
        _, X = _grid((n,) * 3, (-1.0,) * 3, (1.0,) * 3)
        pts = np.stack(X, -1)
        ex = CF.bump_sum_potential(pts, meta["centers"], meta["widths"], meta["amps"], meta["p"])
        errs.append(np.abs(phi - ex).max() / np.abs(ex).max())
    assert errs[1] < 2e-6
    assert errs[0] / errs[1] > 30.0  # spectral phi_star error dominates (> 4th order drop)


def test_full_solve_1d_matches_quadrature_of_the_integral():
    from scipy import integrate

    n, eps, p, c = 81, 0.5, 12, 0.13
    rho = I.radial_bump((n,), eps, p, center=[c])
    h = I.grid_spacing((n,))
    phi = P.solve(rho, h)
    x = -1.0 + h[0] * np.arange(n)
    f = lambda s: (1 - (s - c) ** 2 / eps**2) ** p
    for i in (0, 7, 40, 53, n - 1):
        pts = [x[i]] if c - eps < x[i] < c + eps else None
        ex = integrate.quad(lambda s: 0.5 * abs(x[i] - s) * f(s), c - eps, c + eps, points=pts,
                            epsabs=1e-14, epsrel=1e-14, limit=200)[0]
        assert abs(phi[i] - ex) < 1e-9


def test_discrete_poisson_relation_decays_at_fourth_order():
    # L_h phi - (rho + sum_i h_i^2/12 D2_i rho) = O(h^4) at interior nodes
    # (eq. 4thOrderRelation2D); checked on the full solution of a 2D bump.
    res = []
    for n in (65, 129):
        rho, h, _ = I.workload_bumps((n, n), seed=9)
        phi = P.solve(rho, h, 6)
        lhs = P.apply_Lh(phi, h)
        rhs = rho[1:-1, 1:-1] + sum(
            h[i] ** 2 / 12.0 * P._restrict(P.d2(rho, i, h[i]), [0 if a == i else 1 for a in range(2)])
            for i in range(2)
        )
        res.append(np.abs(lhs - rhs)[3:-3, 3:-3].max())
    assert res[0] / res[1] > 12.0


# ---------------------------------------------------------------------------
# Adjoint of the whole map rho -> phi
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,h", [((9,), (0.2,)), ((9, 11), (0.2, 0.13)), ((12, 13), (0.1, 0.07)),
                                     ((8, 9, 10), (0.2, 0.17, 0.11)), ((10, 11, 12), (0.1, 0.12, 0.09))])
@pytest.mark.parametrize("order", [4, 6])
def test_adjoint_dot_product(shape, h, order):
    rng = np.random.default_rng(hash((shape, order)) % 2**32)
    v = rng.standard_normal(shape)
    w = rng.standard_normal(shape)
    lhs = np.sum(P.solve(v, h, order) * w)
    rhs = np.sum(v * P.adjoint(w, h, order))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("shape,h,order", [((8, 9), (0.2, 0.15), 6), ((6, 7), (0.3, 0.2), 4),
                                           ((8, 8, 9), (0.2, 0.25, 0.15), 6)])
def test_adjoint_is_the_transpose_of_the_dense_map(shape, h, order):
    # columns of A from unit vectors on the interior (boundary entries of rho are ignored)
    nI = int(np.prod([s - 2 for s in shape]))
    inner = (slice(1, -1),) * len(shape)
    A = np.zeros((int(np.prod(shape)), nI))
    for c in range(nI):
        e = np.zeros(shape)
        e[inner].flat[c] = 1.0
        A[:, c] = P.solve(e, h, order).ravel()
    rng = np.random.default_rng(1)
    w = rng.standard_normal(shape)
    ref = A.T @ w.ravel()
    got = P.adjoint(w, h, order)
    assert np.abs(got[inner].ravel() - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(got[P.boundary_mask(shape)] == 0.0)


def test_adjoint_pieces_are_transposes():
    # each transposed building block against its forward counterpart
    rng = np.random.default_rng(4)
    h = np.array([0.2, 0.13, 0.17])
    u = rng.standard_normal((9, 10, 11))
    y = rng.standard_normal((7, 8, 9))
    assert abs(np.sum(P.apply_Lh(u, h) * y) - np.sum(u * P.apply_Lh_T(y, h))) < 1e-10
    core = rng.standard_normal((5, 6, 7))
    R = rng.standard_normal((7, 8, 9))
    assert abs(np.sum(P.extrapolate(core) * R) - np.sum(core * P.extrapolate_T(R))) < 1e-11
    cb = rng.standard_normal((5, 6, 7))
    assert abs(np.sum(P.rhs6_core(u, h) * cb) - np.sum(u * P.rhs6_core_T(cb, h))) < 1e-6 * np.abs(P.rhs6_core(u, h)).max()
    rho = rng.standard_normal((9, 10, 11))
    lam = np.where(P.boundary_mask(rho.shape), rng.standard_normal(rho.shape), 0.0)
    lhs = np.sum(P.boundary_values(rho, h) * lam)
    rhs = np.sum(rho[1:-1, 1:-1, 1:-1] * P.boundary_values_T(lam, h)[1:-1, 1:-1, 1:-1])
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
