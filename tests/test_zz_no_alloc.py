"""ips_execute_static: the solve in the library's static device scratch, with
no allocation, against ips_execute on the same plans (bitwise: same kernels,
same order), on two calls in a row with the second grid smaller, and the
size limit of the scratch."""
import ctypes
import gc

import pytest
import torch

from paper_2108_11871_amd import _lib, api
from paper_2108_11871_amd import inputs as I

pytestmark = pytest.mark.gpu


def _live():
    n = ctypes.c_size_t()
    _lib.check(_lib.lib().ips_live_device_bytes(ctypes.byref(n)))
    return n.value


def _static(plan, rho, out, stream):
    return _lib.lib().ips_execute_static(plan._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(stream.cuda_stream))


def _case(shape, seed, precision, scale):
    rho, h, _ = I.workload_bumps(shape, seed=seed, scale=scale)
    return torch.from_numpy(rho).to("cuda:0"), h


def test_static_scratch_matches_execute_on_two_calls():
    from gpu_util import banner

    gc.collect()
    stream = torch.cuda.current_stream()
    cases = [((65, 70, 61), 31, "fp64", [1.0, 1.1, 0.95]),
             ((40, 45, 37), 32, "mixed_fp32_slices", [0.9, 1.0, 1.2])]
    plans, rhos, refs, outs = [], [], [], []
    for shape, seed, prec, scale in cases:
        rho, h = _case(shape, seed, prec, scale)
        own = api.Plan(shape, h, order=6, precision=prec)
        ref = own(rho)
        # tables only: the static call must not need a workspace of the plan
        p = api.Plan(shape, h, order=6, precision=prec, no_workspace=True)
        assert p.workspace_bytes <= _lib.IPS_STATIC_SCRATCH_BYTES
        plans.append((own, p))
        rhos.append(rho)
        refs.append(ref)
        outs.append(torch.full_like(rho, float("nan")))
    torch.cuda.synchronize()
    live = _live()
    torch_bytes = torch.cuda.memory_allocated()
    # two calls in a row, the second with the smaller grid
    for (own, p), rho, out, (shape, _, prec, _) in zip(plans, rhos, outs, cases):
        banner("ips_execute_static %s %s" % (shape, prec))
        assert _static(p, rho, out, stream) == 0, _lib.detail()
    torch.cuda.synchronize()
    assert _live() == live                        # the library allocated nothing
    assert torch.cuda.memory_allocated() == torch_bytes
    for out, ref in zip(outs, refs):
        assert torch.equal(out, ref)
    # the plan-owned path still works after the static calls (no binding changed)
    own, p = plans[1]
    with pytest.raises(_lib.IpsError):
        p(rhos[1])  # a no-workspace plan still has none
    again = own(rhos[1])
    torch.cuda.synchronize()
    assert torch.equal(again, refs[1])
    # a plan with its own workspace gives the same through the static call
    out = torch.empty_like(rhos[0])
    assert _static(plans[0][0], rhos[0], out, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, refs[0])
    for own, p in plans:
        own.close()
        p.close()


def test_static_scratch_rejects_large_plans():
    from gpu_util import banner

    banner("ips_execute_static size limit")
    shape = (129, 129, 129)
    h = [2.0 / 128] * 3
    p = api.Plan(shape, h, order=6, no_workspace=True)
    assert p.workspace_bytes > _lib.IPS_STATIC_SCRATCH_BYTES
    rho = torch.zeros(shape, dtype=torch.float64, device="cuda:0")
    out = torch.empty_like(rho)
    rc = _static(p, rho, out, torch.cuda.current_stream())
    assert rc == -5
    assert "static scratch" in _lib.detail()
    p.close()
