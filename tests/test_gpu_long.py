"""Transforms longer than 2048 points (1D and 2D grids up to 4097 nodes per
axis): one complex sequence per LDS tile, twiddles from global memory,
1024-thread blocks.

* full parity with the FP64 oracle (1e-12) where the oracle finishes in
  seconds: 1D up to 4097 nodes, 2D with one long axis, 2049^2 (length-4096
  transforms on both axes), a non-power-of-two length (3001 nodes: 6000 =
  2^4 3 5^3), forward and adjoint;
* 2D 4097^2 (length-8192 transforms), the differentiation workload: boundary
  values at sampled nodes against the oracle's direct sums, error against
  the closed-form potential at sampled nodes, mixed modes against FP64, the
  dot-product identity of forward and adjoint, and gradients of
  J = 1/2 |phi(rho) - phi_target|^2 against central differences.
"""
import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import poisson as P
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _fwd(rho, h, order, precision="fp64"):
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    plan = api.Plan(rho.shape, h, order=order, precision=precision)
    out = plan(to_dev(rho))
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    plan.close()
    return res


def _adj(w, h, order):
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    plan = api.Plan(w.shape, h, order=order)
    out = plan.adjoint(to_dev(w))
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("n", [2049, 3001, 4097])
def test_1d_long(n):
    from gpu_util import banner, rel_err

    rho = I.radial_bump((n,), 0.5, 8, center=[0.1])
    h = I.grid_spacing((n,))
    err = rel_err(_fwd(rho, h, 4), P.solve(rho, h, 4))
    w = np.random.default_rng(n).standard_normal(n)
    aerr = rel_err(_adj(w, h, 4), P.adjoint(w, h, 4))
    banner("1D n=%d: forward %.2e adjoint %.2e" % (n, err, aerr))
    assert err < TOL and aerr < TOL


@pytest.mark.parametrize("shape,order", [((4097, 41), 6), ((37, 4097), 6), ((3001, 65), 4),
                                         ((2049, 2049), 6)])
def test_2d_long_matches_oracle(shape, order):
    from gpu_util import banner, rel_err

    rho, h, _ = I.workload_bumps(shape, seed=7, scale=[1.0, 1.2])
    boundary = "fft" if min(shape) > 1000 else "direct"
    err = rel_err(_fwd(rho, h, order), P.solve(rho, h, order, boundary=boundary))
    banner("2D %s order %d: forward rel err %.2e" % (shape, order, err))
    assert err < TOL
    if min(shape) < 100:
        w = np.random.default_rng(3).standard_normal(shape)
        aerr = rel_err(_adj(w, h, order), P.adjoint(w, h, order))
        banner("  adjoint rel err %.2e" % aerr)
        assert aerr < TOL


@pytest.mark.parametrize("mode", ["mixed_fp32", "mixed_fp32_slices"])
def test_2d_long_mixed(mode):
    from gpu_util import rel_err

    rho, h, _ = I.workload_bumps((4097, 41), seed=7)
    assert rel_err(_fwd(rho, h, 6, mode), _fwd(rho, h, 6)) < 1e-6


def test_2d_4097_forward_backward():
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import banner, to_dev

    n = 4097
    rho, h, meta = I.workload_bumps((n, n), seed=7)
    rho_d = to_dev(rho)
    plan = api.Plan(rho.shape, h, order=6)
    phi_d = plan(rho_d)
    torch.cuda.synchronize()
    phi = phi_d.cpu().numpy()
    rng = np.random.default_rng(41)
    M = n - 1
    tg = [(0, 0), (0, M), (M, 0), (M, M), (0, M // 2), (M, M // 2), (M // 2, 0), (M // 2, M)]
    for _ in range(200):
        j = int(rng.integers(0, n))
        tg.append((0, j) if rng.random() < 0.25 else (M, j) if rng.random() < 0.33 else
                  (j, 0) if rng.random() < 0.5 else (j, M))
    tg = np.array(tg, dtype=np.int64)
    g_ref = P.boundary_values_at(rho, h, tg)
    gerr = float(np.abs(phi[tg[:, 0], tg[:, 1]] - g_ref).max() / np.abs(g_ref).max())
    idx = rng.integers(0, n, (100000, 2))
    x = -1.0 + h[0] * idx
    ex = CF.bump_sum_potential(x, meta["centers"], meta["widths"], meta["amps"], meta["p"])
    cerr = float(np.abs(phi[idx[:, 0], idx[:, 1]] - ex).max() / np.abs(ex).max())
    banner("2D 4097^2: boundary samples %.2e, closed form at samples %.2e" % (gerr, cerr))
    assert gerr < TOL
    assert cerr < 1e-10
    for mode in ("mixed_fp32", "mixed_fp32_slices"):
        pm = api.Plan(rho.shape, h, order=6, precision=mode)
        merr = float((pm(rho_d) - phi_d).abs().max() / phi_d.abs().max())
        pm.close()
        banner("  %s vs FP64 %.2e" % (mode, merr))
        assert merr < 1e-6
    # backward: dot-product identity and gradients against central differences
    g = torch.Generator(device="cuda:0").manual_seed(8)
    v = torch.randn(rho.shape, dtype=torch.float64, device="cuda:0", generator=g)
    w = torch.randn(rho.shape, dtype=torch.float64, device="cuda:0", generator=g)
    Av, Atw = plan(v), plan.adjoint(w)
    lhs = float((Av * w).sum())
    rhs = float((v[1:-1, 1:-1] * Atw[1:-1, 1:-1]).sum())
    scale = float((Av.abs() * w.abs()).sum())
    banner("  <Av,w> %.15e <v,A^T w> %.15e rel %.2e" % (lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-12 * scale
    tgt, _, _ = I.workload_bumps((n, n), seed=5)
    target = plan(to_dev(tgt)).detach()
    r = rho_d.clone().requires_grad_(True)
    J = 0.5 * ((api.SolveFn.apply(r, plan) - target) ** 2).sum()
    J.backward()
    grad = r.grad.detach()

    def Jof(x):
        with torch.no_grad():
            return 0.5 * float(((plan(x) - target) ** 2).sum())

    for t in range(4):
        if t % 2 == 0:
            vv = to_dev(I.workload_bumps((n, n), seed=300 + t)[0])
        else:
            vv = torch.zeros_like(rho_d)
            vv[1:-1, 1:-1] = torch.randn((n - 2, n - 2), dtype=torch.float64, device="cuda:0", generator=g)
        tau = float(rho_d.abs().max() / vv.abs().max())
        fd = (Jof(rho_d + tau * vv) - Jof(rho_d - tau * vv)) / (2.0 * tau)
        an = float((grad * vv).sum())
        rel = abs(fd - an) / max(abs(fd), abs(an))
        banner("  direction %d: <grad,v> %.12e FD %.12e rel %.2e" % (t, an, fd, rel))
        assert rel < 1e-10
    plan.close()
