"""Python binding of the HIP solver: torch tensors in, torch tensors out.

Only argument marshalling happens here: tensors provide device memory and the
current HIP stream, every arithmetic step runs in libipoisson.so.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib
from ._lib import (IPS_FLAG_ADJOINT, IPS_FLAG_AUTOTUNE, IPS_FLAG_BATCH_EAGER, IPS_FLAG_BATCH_SMOOTH,
                   IPS_FLAG_NO_WORKSPACE, IPS_FLAG_SCREEN_DIRECT,
                   IPS_FLAG_SCREENING, IPS_FLAG_STAGE_TIMING, IPS_FP64, IPS_MIXED_FP32, IPS_MIXED_FP32_SLICES, STAGES, check, f64_array,
                   i64_array, library_path, lib)

PRECISIONS = {"fp64": IPS_FP64, "mixed_fp32": IPS_MIXED_FP32,
              "mixed_fp32_slices": IPS_MIXED_FP32_SLICES}

__all__ = ["solve", "release_solve_cache", "solve_cache_size", "Plan", "Batch", "SolveFn", "PRECISIONS",
           "library_path", "extension"]


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_grid(t: torch.Tensor):
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError("rho must be float64")
    if not t.is_cuda:
        raise ValueError("rho must live on a GPU device")
    if not t.is_contiguous():
        raise ValueError("rho must be contiguous (row-major, last axis fastest)")
    if t.dim() not in (1, 2, 3):
        raise ValueError("rho must have 1, 2 or 3 dimensions")


def _check_out(out: torch.Tensor, like: torch.Tensor, name: str = "out"):
    """A caller-supplied output must match the input exactly: the library writes
    prod(shape) doubles through its pointer."""
    if not isinstance(out, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if out.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if out.device != like.device:
        raise ValueError("%s must live on %s" % (name, like.device))
    if tuple(out.shape) != tuple(like.shape):
        raise ValueError("%s shape %s does not match %s" % (name, tuple(out.shape), tuple(like.shape)))
    if not out.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def extension(shape: Sequence[int], margin):
    """(extended shape, offset of the caller's node 0) of an extended solve
    (ips_extension): each axis grows by 2 margin nodes, then to the next panel
    count with no prime factor above 5."""
    shape = tuple(int(v) for v in shape)
    d = len(shape)
    mm = list(margin) if hasattr(margin, "__len__") else [int(margin)] * d
    if len(mm) != d:
        raise ValueError("margin needs one entry per axis")
    ne = (ctypes.c_int64 * d)()
    off = (ctypes.c_int64 * d)()
    check(lib().ips_extension(d, i64_array(shape), i64_array(mm), ne, off))
    return tuple(ne), tuple(off)


class Plan:
    """A reusable solve of one grid geometry (ips_plan_create / ips_execute)."""

    def __init__(self, shape: Sequence[int], h, order: int = 6, precision: str = "fp64",
                 device=None, timing: bool = False, adjoint: bool = False, autotune: bool = False,
                 margin=None, no_workspace: bool = False, screening: bool = False,
                 screen_direct: bool = False):
        """margin: None, or nodes added on each side of every axis (an int or one
        per axis); the solve then runs on the enlarged grid of `extension` and
        returns phi at the caller's nodes (ips_plan_create_extended).
        no_workspace: create the plan without an execution workspace; bind one
        with `set_workspace` before the first solve (IPS_FLAG_NO_WORKSPACE).
        screening: boundary values from the screening charge d phi*/dn and a
        corrected surface quadrature instead of the volume sums
        (IPS_FLAG_SCREENING; FP64, no adjoint).
        screen_direct: with screening, the 3D surface sums by direct summation
        instead of by transforms (IPS_FLAG_SCREEN_DIRECT: no tables, O(n^4))."""
        self.shape = tuple(int(v) for v in shape)
        d = len(self.shape)
        hh = list(h) if hasattr(h, "__len__") else [float(h)] * d
        if len(hh) != d:
            raise ValueError("h needs one entry per axis")
        self.h = tuple(float(v) for v in hh)
        self.order = int(order)
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        handle = ctypes.c_void_p()
        flags = ((IPS_FLAG_STAGE_TIMING if timing else 0) | (IPS_FLAG_ADJOINT if adjoint else 0)
                 | (IPS_FLAG_AUTOTUNE if autotune else 0) | (IPS_FLAG_NO_WORKSPACE if no_workspace else 0)
                 | (IPS_FLAG_SCREENING if screening else 0) | (IPS_FLAG_SCREEN_DIRECT if screen_direct else 0))
        self.margin = None
        with torch.cuda.device(self.device):
            if margin is None:
                check(lib().ips_plan_create(ctypes.byref(handle), d, i64_array(self.shape),
                                            f64_array(self.h), self.order, PRECISIONS[precision], flags))
            else:
                mm = list(margin) if hasattr(margin, "__len__") else [int(margin)] * d
                if len(mm) != d:
                    raise ValueError("margin needs one entry per axis")
                self.margin = tuple(int(v) for v in mm)
                check(lib().ips_plan_create_extended(ctypes.byref(handle), d, i64_array(self.shape),
                                                     f64_array(self.h), self.order, PRECISIONS[precision],
                                                     flags, i64_array(self.margin)))
        self._h = handle

    @property
    def workspace_bytes(self) -> int:
        """Bytes of execution workspace the plan needs (ips_plan_workspace_size)."""
        n = ctypes.c_size_t()
        check(lib().ips_plan_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    @property
    def table_bytes(self) -> int:
        """Bytes of tables (kernel spectra, twiddles, ...) held by the plan."""
        n = ctypes.c_size_t()
        check(lib().ips_plan_table_size(self._h, ctypes.byref(n)))
        return n.value

    def set_workspace(self, buf: torch.Tensor | None, nbytes: int | None = None):
        """Run in caller-owned device memory (ips_plan_set_workspace); None returns
        to a plan-owned workspace.  The tensor must stay alive while solves of
        this plan are enqueued; nbytes defaults to the tensor's size."""
        if buf is None:
            check(lib().ips_plan_set_workspace(self._h, None, 0))
            self._ws = None
            return
        if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("the workspace must be a contiguous GPU tensor")
        size = buf.numel() * buf.element_size() if nbytes is None else int(nbytes)
        if size > buf.numel() * buf.element_size():
            raise ValueError("nbytes exceeds the tensor")
        with torch.cuda.device(buf.device):
            check(lib().ips_plan_set_workspace(self._h, ctypes.c_void_p(buf.data_ptr()), size))
        self._ws = buf

    def __call__(self, rho: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_grid(rho)
        if tuple(rho.shape) != self.shape:
            raise ValueError("rho shape %s does not match the plan %s" % (tuple(rho.shape), self.shape))
        if out is None:
            out = torch.empty_like(rho)
        else:
            _check_out(out, rho)
        with torch.cuda.device(rho.device):
            check(lib().ips_execute(self._h, ctypes.c_void_p(rho.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(_stream_handle(rho.device))))
        return out

    def adjoint(self, phi_bar: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """rho_bar = A^T phi_bar for the map A: rho -> phi of this plan (FP64 data;
        mixed plans run the volume sine transforms in FP32 tiles)."""
        _check_grid(phi_bar)
        if tuple(phi_bar.shape) != self.shape:
            raise ValueError("phi_bar shape %s does not match the plan %s" % (tuple(phi_bar.shape), self.shape))
        if out is None:
            out = torch.empty_like(phi_bar)
        else:
            _check_out(out, phi_bar)
        with torch.cuda.device(phi_bar.device):
            check(lib().ips_execute_adjoint(self._h, ctypes.c_void_p(phi_bar.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(_stream_handle(phi_bar.device))))
        return out

    def stage_times(self) -> dict:
        """{stage name: (total ms, executions)} since the last reset (timing plans only)."""
        out = {}
        for i, name in enumerate(STAGES):
            ms = ctypes.c_double()
            calls = ctypes.c_int64()
            check(lib().ips_plan_stage_time(self._h, i, ctypes.byref(ms), ctypes.byref(calls)))
            out[name] = (ms.value, calls.value)
        return out

    def reset_stage_times(self):
        check(lib().ips_plan_reset_stage_times(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ips_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(rho: torch.Tensor, h, order: int = 6, precision: str = "fp64") -> torch.Tensor:
    """phi = G * rho on the grid of rho (blocking ips_solve_ex on the null stream,
    with the library's plan cache)."""
    _check_grid(rho)
    if precision not in PRECISIONS:
        raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
    d = rho.dim()
    hh = list(h) if hasattr(h, "__len__") else [float(h)] * d
    if len(hh) != d:
        raise ValueError("h needs one entry per axis")
    out = torch.empty_like(rho)
    torch.cuda.current_stream(rho.device).synchronize()
    with torch.cuda.device(rho.device):
        check(lib().ips_solve_ex(d, i64_array(rho.shape), f64_array(hh),
                                 ctypes.c_void_p(rho.data_ptr()), int(order), PRECISIONS[precision],
                                 ctypes.c_void_p(out.data_ptr())))
    return out


def release_solve_cache():
    """Destroy the idle plans of the solve cache (ips_solve_release_cache)."""
    check(lib().ips_solve_release_cache())


def solve_cache_size() -> int:
    n = ctypes.c_size_t()
    check(lib().ips_solve_cache_size(ctypes.byref(n)))
    return n.value


class Batch:
    """Many independent problems of uneven size (ips_batch_create / ips_batch_execute)."""

    def __init__(self, shapes, hs, order: int = 6, precision: str = "fp64", eager: bool = False,
                 autotune: bool = False, device=None, smooth: bool = False, screening: bool = False):
        """smooth: solve every problem on its 5-smooth extension (IPS_FLAG_BATCH_SMOOTH);
        screening: boundary values from the screening charge (IPS_FLAG_SCREENING)."""
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        count = len(self.shapes)
        dims = (ctypes.c_int * count)(*[len(s) for s in self.shapes])
        nn = (ctypes.c_int64 * (3 * count))()
        hh = (ctypes.c_double * (3 * count))()
        for b, (s, h) in enumerate(zip(self.shapes, hs)):
            for a in range(len(s)):
                nn[3 * b + a] = s[a]
                hh[3 * b + a] = float(h[a])
        handle = ctypes.c_void_p()
        flags = ((IPS_FLAG_BATCH_EAGER if eager else 0) | (IPS_FLAG_AUTOTUNE if autotune else 0)
                 | (IPS_FLAG_BATCH_SMOOTH if smooth else 0) | (IPS_FLAG_SCREENING if screening else 0))
        with torch.cuda.device(self.device):
            check(lib().ips_batch_create(ctypes.byref(handle), count, dims, nn, hh, int(order),
                                         PRECISIONS[precision], flags))
        self._h = handle
        self.count = count

    def __call__(self, rhos, outs=None):
        if len(rhos) != self.count:
            raise ValueError("expected %d right-hand sides" % self.count)
        for r, s in zip(rhos, self.shapes):
            _check_grid(r)
            if tuple(r.shape) != s:
                raise ValueError("rho shape %s does not match %s" % (tuple(r.shape), s))
        if outs is None:
            outs = [torch.empty_like(r) for r in rhos]
        else:
            if len(outs) != self.count:
                raise ValueError("expected %d outputs" % self.count)
            for o, r in zip(outs, rhos):
                _check_out(o, r, "outs[i]")
        dev = rhos[0].device
        for r in rhos:
            if r.device != dev:
                raise ValueError("every problem of a batch must live on one device")
        rp = (ctypes.c_void_p * self.count)(*[r.data_ptr() for r in rhos])
        pp = (ctypes.c_void_p * self.count)(*[o.data_ptr() for o in outs])
        with torch.cuda.device(dev):
            check(lib().ips_batch_execute(self._h, rp, pp, ctypes.c_void_p(_stream_handle(dev))))
        return outs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ips_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SolveFn(torch.autograd.Function):
    """phi = A rho with dJ/drho = A^T dJ/dphi (A^T runs in the HIP adjoint)."""

    @staticmethod
    def forward(ctx, rho, plan: Plan):
        ctx.plan = plan
        return plan(rho.contiguous())

    @staticmethod
    def backward(ctx, grad_phi):
        return ctx.plan.adjoint(grad_phi.contiguous()), None
