"""Automatic domain extension (ips_extension / ips_plan_create_extended):
the caller's grid is placed inside an enlarged box (a margin on every side,
then panel counts with no prime factor above 5) and phi is returned at the
caller's nodes (Section 2: the support of rho must lie a distance sigma
inside the box, and the panel counts must suit the FFT).

Bars:
* FP64 against the oracle solved on the explicitly enlarged grid and cropped:
  1e-12 relative, max norm (rho is nonzero up to the caller's boundary: those
  nodes are interior in the enlarged box);
* the adjoint of the extended map by the dot-product identity: 1e-12;
* mixed precision within 1e-6 of FP64;
* a bump well inside the caller's box: the extended solve agrees with the
  plain one to the method's accuracy (the solution does not depend on the box).
"""
import numpy as np
import pytest

from oracle import poisson as P
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu


def _oracle_extended(rho, h, order, margin):
    from paper_2108_11871_amd import api

    ne, off = api.extension(rho.shape, margin)
    big = np.zeros(ne)
    sl = tuple(slice(o, o + s) for o, s in zip(off, rho.shape))
    big[sl] = rho
    return P.solve(big, h, order)[sl]


@pytest.mark.parametrize("shape,h,order,margin", [
    ((20, 17), (0.1, 0.12), 4, (3, 2)),
    ((20, 17), (0.1, 0.12), 6, (3, 2)),
    ((33, 30), (0.05, 0.06), 6, 4),
    ((12, 10, 14), (0.1, 0.12, 0.09), 6, 2),
    ((9, 11, 10), (0.2, 0.17, 0.15), 4, (1, 3, 0)),
])
def test_extended_solve_matches_oracle(shape, h, order, margin):
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import banner, rel_err, to_dev

    banner("extended shape=%s order=%d margin=%s" % (shape, order, margin))
    rho = np.random.default_rng(sum(shape) + order).standard_normal(shape)
    ref = _oracle_extended(rho, h, order, margin)
    plan = api.Plan(shape, h, order=order, margin=margin)
    got = plan(to_dev(rho))
    torch.cuda.synchronize()
    err = rel_err(got.cpu().numpy(), ref)
    plan.close()
    print("  rel err %.3e" % err, flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("shape,margin", [((40, 33), 5), ((24, 20, 22), 3)])
def test_extended_adjoint_dot_product(shape, margin):
    import torch
    from paper_2108_11871_amd import api

    h = tuple(1.0 / (s - 1) for s in shape)
    plan = api.Plan(shape, h, order=6, margin=margin)
    g = torch.Generator(device="cuda:0").manual_seed(3)
    v = torch.randn(shape, dtype=torch.float64, device="cuda:0", generator=g)
    w = torch.randn(shape, dtype=torch.float64, device="cuda:0", generator=g)
    lhs = float((plan(v) * w).sum())
    rhs = float((v * plan.adjoint(w)).sum())
    scale = float((plan(v).abs() * w.abs()).sum())
    plan.close()
    print("  <Av,w> %.15e  <v,A^T w> %.15e" % (lhs, rhs), flush=True)
    assert abs(lhs - rhs) <= 1e-12 * scale


def test_extended_mixed_within_1e6_of_fp64():
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    shape = (65, 65, 65)
    rho, h = I.radial_bump(shape, 0.6, 10), I.grid_spacing(shape)
    r = to_dev(rho)
    ref = api.Plan(shape, h, order=6, margin=6)(r)
    for mode in ("mixed_fp32", "mixed_fp32_slices"):
        got = api.Plan(shape, h, order=6, precision=mode, margin=6)(r)
        torch.cuda.synchronize()
        err = float((got - ref).abs().max() / ref.abs().max())
        print("  %s rel err %.2e" % (mode, err), flush=True)
        assert err < 1e-6


def test_extension_leaves_the_solution_unchanged():
    """A bump well inside the box: enlarging the box changes phi at the
    caller's nodes only at the level of the method's error."""
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    shape = (65, 65, 65)
    rho, h = I.radial_bump(shape, 0.6, 10), I.grid_spacing(shape)  # support 0.4 inside the box
    r = to_dev(rho)
    plain = api.Plan(shape, h, order=6)(r)
    ext = api.Plan(shape, h, order=6, margin=12)(r)
    torch.cuda.synchronize()
    err = float((ext - plain).abs().max() / plain.abs().max())
    print("  extended vs plain rel diff %.2e" % err, flush=True)
    assert err < 1e-6
