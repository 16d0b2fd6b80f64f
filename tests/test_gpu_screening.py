"""Screening-charge boundary values on the GPU (IPS_FLAG_SCREENING) against the
oracle's screening reading (oracle/screening.py), node by node at 1e-12
relative to max |phi|: 1D, 2D and 3D (up to 65x60x70, where the surface sums
run by transforms with several row groups), orders 4 and 6, anisotropic
spacings, ragged sizes; the transforms against the direct sums up to 257^3;
plus the variant's rejections (mixed precision, adjoint)."""
import numpy as np
import pytest
import torch

from oracle import screening as S
from paper_2108_11871_amd import _lib, api
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _run(shape, order, seed, scale):
    from gpu_util import banner, rel_err, to_dev

    banner("screening %s order %d seed %d" % (shape, order, seed))
    rho, h, _ = I.workload_bumps(shape, seed=seed, scale=scale)
    plan = api.Plan(shape, h, order=order, screening=True)
    got = plan(to_dev(rho)).cpu().numpy()
    plan.close()
    ref = S.solve_screening(rho, h, order)
    err = rel_err(got, ref)
    banner("  rel err vs the oracle %.3e" % err)
    assert err <= TOL
    return got, rho, h


@pytest.mark.parametrize("n", [9, 65, 257, 1025])
def test_screening_1d(n):
    _run((n,), 4, 3, [1.0])


@pytest.mark.parametrize("shape,order", [((65, 71), 4), ((40, 33), 6), ((129, 97), 6), ((7, 9), 4)])
def test_screening_2d(shape, order):
    _run(shape, order, 4, [1.0, 1.2])


@pytest.mark.parametrize("shape,order", [((25, 28, 23), 6), ((33, 33, 33), 4), ((17, 20, 31), 6), ((8, 9, 10), 6),
                                         ((65, 60, 70), 6)])
def test_screening_3d(shape, order):
    _run(shape, order, 5, [1.0, 0.9, 1.15])


@pytest.mark.parametrize("shape", [(41, 37, 45), (65, 65, 65), (9, 30, 12), (129, 129, 129), (150, 20, 41),
                                   (257, 257, 257), (330, 12, 20), (20, 400, 16)])
def test_screening_transforms_match_the_direct_sums(shape):
    """The 3D surface sums by transforms (the default) against the direct sums
    of IPS_FLAG_SCREEN_DIRECT, on the same input: one and several row groups
    per wavenumber, one and several table tiles per group, thin boxes, and the
    bench grid (the direct sums are pinned to the oracle on the smaller grids).
    Face sides up to 320 nodes run the perpendicular sums on the matrix cores,
    longer ones (the last two shapes) on the vector units."""
    from gpu_util import banner, rel_err, to_dev

    banner("screening transforms vs direct %s" % (shape,))
    rho, h, _ = I.workload_bumps(shape, seed=21, scale=[1.0, 1.1, 0.95])
    x = to_dev(rho)
    pf = api.Plan(shape, h, order=6, screening=True)
    pd = api.Plan(shape, h, order=6, screening=True, screen_direct=True)
    fast = pf(x).cpu().numpy()
    direct = pd(x).cpu().numpy()
    pf.close()
    pd.close()
    err = rel_err(fast, direct)
    banner("  rel err %.3e" % err)
    assert err <= TOL


def test_screening_boundary_values_are_the_surface_sums():
    """The boundary nodes of the GPU result are the oracle's surface sums g."""
    from gpu_util import to_dev

    shape = (30, 27, 33)
    rho, h, _ = I.workload_bumps(shape, seed=12, scale=[1.0, 1.05, 0.95])
    plan = api.Plan(shape, h, order=6, screening=True)
    got = plan(to_dev(rho)).cpu().numpy()
    plan.close()
    g = S.screening_boundary_values(rho, h)
    from oracle import poisson as P

    m = P.boundary_mask(shape)
    assert np.abs(got[m] - g[m]).max() <= TOL * np.abs(g[m]).max()


def test_screening_rejections():
    L = _lib.lib()
    import ctypes

    hnd = ctypes.c_void_p()
    n = _lib.i64_array([20, 20, 20])
    h = _lib.f64_array([0.1] * 3)
    assert L.ips_plan_create(ctypes.byref(hnd), 3, n, h, 6, 1, 32) == -2  # mixed precision
    assert L.ips_plan_create(ctypes.byref(hnd), 3, n, h, 6, 0, 32 | 2) == -2  # adjoint flag
    assert L.ips_plan_create(ctypes.byref(hnd), 3, n, h, 6, 0, 128) == -1  # direct sums without screening
    p = api.Plan((20, 20, 20), [0.1] * 3, screening=True)
    x = torch.zeros((20, 20, 20), dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.IpsError) as ei:
        p.adjoint(x)
    assert ei.value.status == -2
    p.close()
