"""Plan memory through the C ABI: caller-supplied workspaces
(ips_plan_set_workspace, IPS_FLAG_NO_WORKSPACE), the ips_solve plan cache
with a precision (ips_solve_ex), and allocation failures during plan creation
(IPS_TEST_FAIL_ALLOC) that must leave no device memory behind."""
import ctypes
import os

import numpy as np
import pytest
import torch

from paper_2108_11871_amd import _lib, api
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu


def _live():
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().ips_live_device_bytes(ctypes.byref(n)))
    return n.value


def _rho(shape, seed):
    from gpu_util import to_dev

    rho, h, _ = I.workload_bumps(shape, seed=seed, scale=[1.0, 0.9, 1.2][: len(shape)])
    return to_dev(rho), h


@pytest.mark.parametrize("shape,order,precision", [
    ((33, 40, 37), 6, "fp64"),
    ((33, 40, 37), 6, "mixed_fp32_slices"),
    ((29, 31, 26), 4, "mixed_fp32"),
    ((61, 47), 6, "fp64"),
])
def test_caller_workspace_is_bitwise_identical(shape, order, precision):
    from gpu_util import banner

    banner("caller workspace %s order %d %s" % (shape, order, precision))
    rho, h = _rho(shape, 11)
    own = api.Plan(shape, h, order=order, precision=precision)
    ref = own(rho)
    ext = api.Plan(shape, h, order=order, precision=precision, no_workspace=True)
    need = ext.workspace_bytes
    assert need == own.workspace_bytes > 0
    # a plan without a workspace refuses to run
    with pytest.raises(_lib.IpsError) as ei:
        ext(rho)
    assert ei.value.status == -5
    # too short: IPS_E_WORKSPACE, the plan stays without one
    buf = torch.empty(need // 8 + 64, dtype=torch.float64, device="cuda:0")
    with pytest.raises(_lib.IpsError) as ei:
        ext.set_workspace(buf, need - 8)
    assert ei.value.status == -5
    with pytest.raises(_lib.IpsError):
        ext(rho)
    # garbage in the caller's buffer must not matter
    buf.fill_(float("nan"))
    ext.set_workspace(buf)
    got = ext(rho)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    # a repeated solve in the same buffer
    got2 = ext(rho)
    torch.cuda.synchronize()
    assert torch.equal(got2, ref)
    # back to a plan-owned workspace
    ext.set_workspace(None)
    got3 = ext(rho)
    torch.cuda.synchronize()
    assert torch.equal(got3, ref)
    own.close()
    ext.close()


def test_two_plans_share_one_workspace():
    from gpu_util import banner

    banner("shared workspace 33^3 / 45x40x38")
    ra, ha = _rho((33, 33, 33), 3)
    rb, hb = _rho((45, 40, 38), 4)
    pa = api.Plan(ra.shape, ha, no_workspace=True)
    pb = api.Plan(rb.shape, hb, no_workspace=True)
    need = max(pa.workspace_bytes, pb.workspace_bytes)
    buf = torch.empty(need // 8 + 1, dtype=torch.float64, device="cuda:0")
    pa.set_workspace(buf)
    pb.set_workspace(buf)
    ya = pa(ra)
    yb = pb(rb)  # same stream: runs after the first solve has finished with the buffer
    qa = api.Plan(ra.shape, ha)
    qb = api.Plan(rb.shape, hb)
    torch.cuda.synchronize()
    assert torch.equal(ya, qa(ra))
    assert torch.equal(yb, qb(rb))
    for p in (pa, pb, qa, qb):
        p.close()


def test_adjoint_in_caller_workspace(no_gc):
    from gpu_util import banner

    banner("adjoint in caller workspace 30x33x35")
    rho, h = _rho((30, 33, 35), 5)
    own = api.Plan(rho.shape, h, adjoint=True)
    ext = api.Plan(rho.shape, h, adjoint=True, no_workspace=True)
    assert ext.workspace_bytes == own.workspace_bytes
    plain = api.Plan(rho.shape, h)
    assert ext.workspace_bytes > plain.workspace_bytes  # the adjoint buffers are inside
    buf = torch.empty(ext.workspace_bytes // 8 + 1, dtype=torch.float64, device="cuda:0")
    ext.set_workspace(buf)
    live = _live()
    a = ext.adjoint(rho)
    b = own.adjoint(rho)
    torch.cuda.synchronize()
    assert _live() == live  # nothing allocated by the adjoint
    assert torch.equal(a, b)
    for p in (own, ext, plain):
        p.close()


def test_workspace_rejects_bad_buffers():
    rho, h = _rho((20, 21, 22), 6)
    p = api.Plan(rho.shape, h, no_workspace=True)
    L = _lib.lib()
    buf = torch.empty(p.workspace_bytes // 8 + 64, dtype=torch.float64, device="cuda:0")
    # misaligned
    rc = L.ips_plan_set_workspace(p._h, ctypes.c_void_p(buf.data_ptr() + 8), p.workspace_bytes)
    assert rc == -1
    # host memory
    host = np.zeros(p.workspace_bytes // 8 + 64)
    rc = L.ips_plan_set_workspace(p._h, ctypes.c_void_p(host.ctypes.data & ~255), p.workspace_bytes)
    assert rc == -1
    # NULL with a size
    assert L.ips_plan_set_workspace(p._h, None, 16) == -1
    p.close()


def test_solve_cache_is_bounded_and_takes_a_precision(no_gc):
    from gpu_util import banner
    from oracle import poisson as P

    banner("ips_solve cache")
    api.release_solve_cache()
    assert api.solve_cache_size() == 0
    base = _live()
    shapes = [(20, 21, 22), (23, 22, 21), (24, 20, 26), (18, 19, 20), (21, 21, 21), (22, 24, 20)]
    for k, s in enumerate(shapes):
        rho, h = _rho(s, 20 + k)
        phi = api.solve(rho, h, order=6)
        ref = P.solve(rho.cpu().numpy(), h, 6)
        got = phi.cpu().numpy()
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12
        assert api.solve_cache_size() <= int(os.environ.get("IPS_SOLVE_CACHE", "4"))
        mixed = api.solve(rho, h, order=6, precision="mixed_fp32_slices")
        merr = float((mixed - phi).abs().max() / phi.abs().max())
        assert merr < 1e-6
    api.release_solve_cache()
    assert api.solve_cache_size() == 0
    assert _live() == base
    with pytest.raises(ValueError):
        api.solve(rho, h, precision="fp16")


@pytest.fixture
def no_gc():
    """Live-byte comparisons must not see plans of earlier tests being collected."""
    import gc

    gc.collect()
    gc.disable()
    yield
    gc.enable()


# a 3D plan makes 2 table allocations per axis, 3 kernel-spectrum tables and
# one workspace block: k = 1..10 fail at every stage, k = 11 succeeds
@pytest.mark.parametrize("k", list(range(1, 12)))
def test_failed_plan_creation_frees_everything(k, monkeypatch, no_gc):
    from gpu_util import banner

    banner("IPS_TEST_FAIL_ALLOC=%d" % k)
    torch.cuda.synchronize()
    base = _live()
    L = _lib.lib()
    monkeypatch.setenv("IPS_TEST_FAIL_ALLOC", str(k))
    handle = ctypes.c_void_p()
    rc = L.ips_plan_create(ctypes.byref(handle), 3, _lib.i64_array([24, 26, 28]),
                           _lib.f64_array([0.1, 0.1, 0.1]), 6, 0, 2)
    monkeypatch.delenv("IPS_TEST_FAIL_ALLOC")
    if rc == 0:
        # fewer allocations than k: the plan is whole
        assert k == 11
        assert handle.value
        assert L.ips_plan_destroy(handle) == 0
    else:
        assert rc == -3, (k, rc)
        assert k <= 10
        assert not handle.value
        assert "IPS_TEST_FAIL_ALLOC" in _lib.detail()
    assert _live() == base
