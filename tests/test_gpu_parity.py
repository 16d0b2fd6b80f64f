"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: FP64 results agree with the oracle to 1e-12 relative (max-norm error
over all nodes divided by the max-norm of the oracle's phi).  Sizes span
several tiles with ragged tails, odd and prime panel counts (FFT lengths
with factors 3, 5, 7 and a direct prime stage), anisotropic spacing, and
both orders.
"""
import numpy as np
import pytest

from oracle import poisson as P
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _gpu_solve(rho, h, order, precision="fp64"):
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    plan = api.Plan(rho.shape, h, order=order, precision=precision)
    phi = plan(to_dev(rho))
    torch.cuda.synchronize()
    out = phi.cpu().numpy()
    plan.close()
    return out


def _check(rho, h, order, tol=TOL, boundary="direct"):
    from gpu_util import banner, rel_err

    banner("shape=%s order=%d" % (rho.shape, order))
    ref = P.solve(rho, h, order, boundary=boundary)
    got = _gpu_solve(rho, h, order)
    err = rel_err(got, ref)
    print("  rel err %.3e" % err, flush=True)
    assert err < tol


@pytest.mark.parametrize("n", [3, 4, 9, 33, 101, 257])
def test_1d(n):
    rho = I.radial_bump((n,), 0.5, 8, center=[0.1]) if n > 8 else np.random.default_rng(n).standard_normal(n)
    h = I.grid_spacing((n,))
    _check(rho, h, 4)


def test_2d_single_bump_65():
    rho, h, meta = I.workload_2d_single(65)
    _check(rho, h, 4)


@pytest.mark.parametrize("shape,order", [((9, 9), 4), ((8, 11), 6), ((33, 41), 4), ((33, 41), 6),
                                         ((50, 38), 6), ((129, 97), 6), ((4, 5), 4), ((3, 5), 4)])
def test_2d_shapes(shape, order):
    rho, h, _ = I.workload_bumps(shape, seed=21, scale=[1.0, 1.3])
    _check(rho, h, order)


@pytest.mark.parametrize("shape,order", [((9, 10, 11), 4), ((9, 10, 11), 6), ((17, 19, 21), 6),
                                         ((24, 30, 27), 6), ((33, 33, 33), 4), ((38, 26, 31), 6),
                                         ((4, 5, 6), 4), ((3, 4, 5), 4)])
def test_3d_shapes(shape, order):
    rho, h, _ = I.workload_bumps(shape, seed=22, scale=[1.0, 0.8, 1.2])
    _check(rho, h, order)


def test_3d_65_order6():
    rho, h, _ = I.workload_bumps_3d(65, seed=1)
    _check(rho, h, 6)


def test_3d_129_order6():
    rho, h, _ = I.workload_bumps_3d(129, seed=1)
    _check(rho, h, 6, boundary="fft")


# Transform lengths 2M = 512 and 1024 along single axes (and 256 along the
# others): the kernel instances with compile-time lengths and tile widths, in
# 2D and in thin 3D boxes whose long axis is in turn the axis of the final
# pass, of the convolution pencils and of the last inverse pass.
LONG_AXIS = [((257, 257), 6), ((513, 385), 6), ((20, 513, 24), 6), ((513, 18, 22), 6), ((24, 20, 513), 4),
             ((129, 257, 40), 6)]


@pytest.mark.parametrize("shape,order", LONG_AXIS)
def test_long_axis_lengths(shape, order):
    rho, h, _ = I.workload_bumps(shape, seed=23, scale=[1.0, 1.1, 0.9][:len(shape)])
    _check(rho, h, order, boundary="fft")


@pytest.mark.parametrize("mode", ["mixed_fp32", "mixed_fp32_slices"])
@pytest.mark.parametrize("shape,order", LONG_AXIS[:4])
def test_long_axis_lengths_mixed(shape, order, mode):
    from gpu_util import banner, rel_err

    rho, h, _ = I.workload_bumps(shape, seed=23, scale=[1.0, 1.1, 0.9][:len(shape)])
    banner("mixed %s shape=%s" % (mode, shape))
    err = rel_err(_gpu_solve(rho, h, order, precision=mode), P.solve(rho, h, order, boundary="fft"))
    print("  rel err %.3e" % err, flush=True)
    assert err < 1e-6


def test_random_rho_3d_small():
    # arbitrary data (no smoothness): parity is purely discrete
    rng = np.random.default_rng(5)
    rho = rng.standard_normal((12, 14, 13))
    h = np.array([0.1, 0.13, 0.07])
    _check(rho, h, 6)
    _check(rho, h, 4)


def test_repeat_is_bitwise_deterministic():
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    rho, h, _ = I.workload_bumps_3d(33, seed=3)
    plan = api.Plan(rho.shape, h, order=6)
    r = to_dev(rho)
    a = plan(r).cpu().numpy()
    b = plan(r).cpu().numpy()
    plan.close()
    assert np.array_equal(a, b)


def test_ips_solve_entry_point():
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import rel_err, to_dev

    rho, h, _ = I.workload_bumps((40, 44), seed=8)
    ref = P.solve(rho, h, 6)
    got = api.solve(to_dev(rho), h, order=6).cpu().numpy()
    assert rel_err(got, ref) < TOL


MIXED_TOL = 1e-6


@pytest.mark.parametrize("mode", ["mixed_fp32", "mixed_fp32_slices"])
@pytest.mark.parametrize("shape", [(33, 41), (129, 129), (33, 37, 29), (65, 65, 65)])
def test_mixed_precision_within_1e6(mode, shape):
    from gpu_util import banner, rel_err

    rho, h, _ = I.workload_bumps(shape, seed=2)
    banner("mixed %s shape=%s" % (mode, shape))
    ref = P.solve(rho, h, 6)
    got = _gpu_solve(rho, h, 6, precision=mode)
    err = rel_err(got, ref)
    print("  rel err %.3e" % err, flush=True)
    assert err < MIXED_TOL


def test_mixed_129_order6():
    from gpu_util import rel_err

    rho, h, _ = I.workload_bumps_3d(129, seed=1)
    ref = P.solve(rho, h, 6, boundary="fft")
    for mode in ("mixed_fp32", "mixed_fp32_slices"):
        err = rel_err(_gpu_solve(rho, h, 6, precision=mode), ref)
        print("  %s rel err %.3e" % (mode, err), flush=True)
        assert err < MIXED_TOL


def test_stage_timing_plan_matches_plain_plan():
    import torch
    from paper_2108_11871_amd import api
    from gpu_util import to_dev

    rho, h, _ = I.workload_bumps_3d(33, seed=4)
    r = to_dev(rho)
    a = api.Plan(rho.shape, h, order=6)
    b = api.Plan(rho.shape, h, order=6, timing=True)
    x = a(r)
    y = b(r)
    b(r)
    st = b.stage_times()
    assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    assert st["conv_x"][1] == 2 and st["final"][0] > 0
    b.reset_stage_times()
    assert b.stage_times()["conv_x"][1] == 0
    a.close()
    b.close()
