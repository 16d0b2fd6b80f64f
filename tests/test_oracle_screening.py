"""Pins of the screening-charge oracle (oracle/screening.py), each against
something other than the oracle itself:

* the lattice constant of the 1/r correction: the published square-lattice
  value -4 zeta(1/2) beta(1/2), its independence of the Ewald split and its
  scaling with the mesh width, and the third-order accuracy it gives the
  punctured trapezoidal rule on a Gaussian (exact integral pi^(3/2));
* the log correction h log(h / 2 pi) on int exp(-x^2) log|x| dx =
  -(sqrt(pi)/2)(gamma + log 4);
* the Gregory end weights integrate cubics exactly;
* sigma for a single sine mode of rho, where phi* and its normal derivative
  are known in closed form (sign and 1/L factors of every face);
* Gauss's theorem: the surface sum of sigma equals the charge of rho;
* 1D: the two end values equal the exact potential (a polynomial integral);
* 2D and 3D: the boundary values converge to the closed-form potential of
  bump sums, at the order a corrected surface trapezoidal rule allows.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import poisson as P
from oracle import screening as S
from paper_2108_11871_amd import inputs as I

# published constants: zeta(1/2) and Dirichlet beta(1/2)
ZETA_HALF = -1.4603545088095868
BETA_HALF = 0.6676914571896092


def test_lattice_constant_square_value_and_scaling():
    c = S.lattice_constant(1.0, 1.0)
    assert abs(c - (-4.0 * ZETA_HALF * BETA_HALF)) < 1e-12
    assert abs(S.lattice_constant(0.01, 0.01) - 0.01 * c) < 1e-14
    # symmetric in its arguments, homogeneous of degree 1
    assert abs(S.lattice_constant(0.3, 0.7) - S.lattice_constant(0.7, 0.3)) < 1e-13
    assert abs(S.lattice_constant(0.6, 1.4) - 2.0 * S.lattice_constant(0.3, 0.7)) < 1e-13


@pytest.mark.parametrize("ratio", [1.0, 1.3, 2.5])
def test_corrected_punctured_rule_is_third_order(ratio):
    """int over R^2 of psi(x)/|x| with psi = exp(-|x|^2)(1 + 0.3 x + 0.2 x y):
    the odd terms integrate to zero, the integral is pi^(3/2)."""
    exact = math.pi ** 1.5
    errs = []
    for hb in (0.2, 0.1, 0.05):
        hc = ratio * hb
        mx, my = int(8 / hb) + 1, int(8 / hc) + 1
        m, n = np.meshgrid(np.arange(-mx, mx + 1), np.arange(-my, my + 1), indexing="ij")
        x, y = m * hb, n * hc
        r = np.hypot(x, y)
        psi = np.exp(-(x * x + y * y)) * (1 + 0.3 * x + 0.2 * x * y)
        r[mx, my] = np.inf
        tr = hb * hc * np.sum(psi / r) + S.lattice_constant(hb, hc)
        errs.append(abs(exact - tr))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(r > 2.7 for r in rates), (errs, rates)
    assert errs[-1] < 5e-4


def test_log_correction_is_third_order():
    exact = -math.sqrt(math.pi) / 2 * (np.euler_gamma + math.log(4.0))
    errs = []
    for h in (0.2, 0.1, 0.05):
        j = np.arange(-int(10 / h), int(10 / h) + 1)
        x = j * h
        psi = np.exp(-x * x) * (1 + 0.4 * x)
        keep = j != 0
        tr = h * np.sum(psi[keep] * np.log(np.abs(x[keep]))) + h * math.log(h / (2 * math.pi))
        errs.append(abs(exact - tr))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(r > 2.8 for r in rates), (errs, rates)


def test_gregory_weights_integrate_cubics():
    for M in (6, 7, 11, 40):
        w = S.gregory_weights(M)
        x = np.arange(M + 1) / M
        for k in range(4):
            assert abs(np.sum(w * x ** k) / M - 1.0 / (k + 1)) < 1e-13


def test_sigma_of_a_single_sine_mode():
    """rho = prod sin(pi k_i (x_i - a_i)/L_i): phi* = -rho / q with q = pi^2 sum k^2/L^2,
    so on face x_a = lo the outward derivative is -(pi k_a/L_a)(-1/q) prod_{b != a} sin,
    and on x_a = hi it is (pi k_a/L_a) cos(pi k_a) (-1/q) prod sin."""
    n = (13, 11, 15)
    h = np.array([0.1, 0.13, 0.07])
    M = np.array(n) - 1
    L = M * h
    k = (2, 3, 1)
    xs = [np.arange(n[a]) * h[a] for a in range(3)]
    mesh = np.meshgrid(*xs, indexing="ij")
    rho = np.ones(n)
    for a in range(3):
        rho = rho * np.sin(math.pi * k[a] * mesh[a] / L[a])
    q = sum((math.pi * k[a] / L[a]) ** 2 for a in range(3))
    sig = S.screening_charge(rho, h)
    for a in range(3):
        others = [b for b in range(3) if b != a]
        fm = np.meshgrid(*[xs[b] for b in others], indexing="ij")
        prod = np.sin(math.pi * k[others[0]] * fm[0] / L[others[0]]) * np.sin(
            math.pi * k[others[1]] * fm[1] / L[others[1]])
        d0 = math.pi * k[a] / L[a] / q
        # phi* = -rho/q: d phi*/dx_a = -d0 prod at x_a = lo, where the outward
        # normal -e_a flips the sign; -d0 cos(pi k_a) prod at x_a = hi (normal +e_a)
        lo = d0 * prod
        hi = -d0 * math.cos(math.pi * k[a]) * prod
        assert np.abs(sig[(a, 0)] - lo).max() < 1e-12
        assert np.abs(sig[(a, 1)] - hi).max() < 1e-12


def test_total_screening_charge_equals_the_charge_of_rho():
    """Gauss: the flux of grad phi* through the boundary is the integral of rho."""
    rho, h, _ = I.workload_bumps((41, 45, 37), seed=8, scale=[1.0, 1.1, 0.9])
    sig = S.screening_charge(rho, h)
    tot = 0.0
    for a in range(3):
        others = [b for b in range(3) if b != a]
        W = np.outer(h[others[0]] * S.gregory_weights(rho.shape[others[0]] - 1),
                     h[others[1]] * S.gregory_weights(rho.shape[others[1]] - 1))
        tot += np.sum(W * (sig[(a, 0)] + sig[(a, 1)]))
    charge = rho[1:-1, 1:-1, 1:-1].sum() * np.prod(h)
    assert abs(tot - charge) < 1e-5 * np.abs(rho).sum() * np.prod(h)


def test_1d_end_values_are_the_exact_potential():
    """phi(end) = (1/2) int |end - s| rho(s) ds, rho a polynomial bump on its
    support: integrated exactly by Gauss-Legendre."""
    n = 257
    rho, h, meta = I.workload_bumps((n,), seed=9)
    g = S.screening_boundary_values(rho, h)
    lo, hi = -1.0, 1.0
    xg, wg = np.polynomial.legendre.leggauss(40)
    exact = [0.0, 0.0]
    for c, w, a in zip(meta["centers"][:, 0], meta["widths"], meta["amps"]):
        s = c + w * xg
        f = a * (1 - ((s - c) / w) ** 2) ** meta["p"]
        exact[0] += 0.5 * np.sum(wg * w * np.abs(s - lo) * f)
        exact[1] += 0.5 * np.sum(wg * w * np.abs(s - hi) * f)
    scale = max(abs(exact[0]), abs(exact[1]))
    assert abs(g[0] - exact[0]) < 1e-10 * scale
    assert abs(g[-1] - exact[1]) < 1e-10 * scale


def _closed_form_boundary_error(shape, seed, scale, fn):
    rho, h, meta = I.workload_bumps(shape, seed=seed, scale=scale)
    g = fn(rho, h)
    mask = P.boundary_mask(rho.shape)
    d = len(shape)
    pts = np.stack(np.meshgrid(*[meta["lo"][a] + h[a] * np.arange(shape[a]) for a in range(d)],
                               indexing="ij"), -1)
    ex = CF.bump_sum_potential(pts[mask], meta["centers"], meta["widths"], meta["amps"], meta["p"])
    return float(np.abs(g[mask] - ex).max() / np.abs(ex).max()), h[0]


def test_2d_boundary_values_converge_to_the_closed_form():
    errs, hs = [], []
    for n in (65, 129, 257):
        e, h = _closed_form_boundary_error((n, n + 6), 5, [1.0, 1.1], S.screening_boundary_values)
        errs.append(e)
        hs.append(h)
    rate = float(np.polyfit(np.log(hs), np.log(errs), 1)[0])
    # a corrected surface trapezoidal rule with kinks at the corners: order ~1.7
    assert rate > 1.4, (errs, rate)
    assert errs[-1] < 1e-4
    # the volume quadrature of the paper is spectrally accurate on the same problem
    ev, _ = _closed_form_boundary_error((257, 263), 5, [1.0, 1.1], P.boundary_values)
    assert ev < 1e-3 * errs[-1]


def test_3d_boundary_values_converge_to_the_closed_form():
    errs = []
    for n in (25, 33, 49):
        e, _ = _closed_form_boundary_error((n, n, n), 6, [1.0, 1.0, 1.0], S.screening_boundary_values)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[-1] < 2e-3, errs
