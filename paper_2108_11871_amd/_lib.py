"""ctypes view of the C ABI in include/ipoisson.h (argument marshalling only).

The library is loaded from the package directory.  There is no fallback: if
libipoisson.so is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipoisson.so")

IPS_OK = 0
STATUS = {
    0: "IPS_OK",
    -1: "IPS_E_INVALID_ARG",
    -2: "IPS_E_UNSUPPORTED",
    -3: "IPS_E_NO_MEMORY",
    -4: "IPS_E_DEVICE",
    -5: "IPS_E_WORKSPACE",
}
IPS_FP64 = 0
IPS_MIXED_FP32 = 1
IPS_MIXED_FP32_SLICES = 2
IPS_FLAG_STAGE_TIMING = 1
IPS_FLAG_ADJOINT = 2
IPS_FLAG_AUTOTUNE = 4
IPS_FLAG_BATCH_EAGER = 8
IPS_FLAG_NO_WORKSPACE = 16
IPS_FLAG_SCREENING = 32
IPS_FLAG_BATCH_SMOOTH = 64
IPS_FLAG_SCREEN_DIRECT = 128
IPS_STATIC_SCRATCH_BYTES = 64 << 20
STAGES = ["rho_z", "conv_x", "conv_y", "rho_y", "conv_z", "faces", "shell_gt", "shell_r6",
          "final", "inv_y", "inv_z", "adjoint", "screen"]

# Every exported symbol with (restype, argtypes).
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
SIGNATURES = {
    "ips_solve": (ctypes.c_int, [ctypes.c_int, _i64p, _dp, _vp, ctypes.c_int, _vp]),
    "ips_solve_ex": (ctypes.c_int, [ctypes.c_int, _i64p, _dp, _vp, ctypes.c_int, ctypes.c_int, _vp]),
    "ips_solve_release_cache": (ctypes.c_int, []),
    "ips_solve_cache_size": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "ips_live_device_bytes": (ctypes.c_int, [ctypes.POINTER(ctypes.c_size_t)]),
    "ips_plan_create": (
        ctypes.c_int,
        [ctypes.POINTER(_vp), ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint],
    ),
    "ips_plan_workspace_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ips_plan_table_size": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "ips_plan_set_workspace": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "ips_extension": (ctypes.c_int, [ctypes.c_int, _i64p, _i64p, _i64p, _i64p]),
    "ips_plan_create_extended": (
        ctypes.c_int,
        [ctypes.POINTER(_vp), ctypes.c_int, _i64p, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_uint, _i64p],
    ),
    "ips_execute": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ips_execute_static": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ips_execute_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "ips_plan_destroy": (ctypes.c_int, [_vp]),
    "ips_batch_create": (
        ctypes.c_int,
        [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(ctypes.c_int), _i64p, _dp,
         ctypes.c_int, ctypes.c_int, ctypes.c_uint],
    ),
    "ips_batch_execute": (ctypes.c_int, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
    "ips_batch_destroy": (ctypes.c_int, [_vp]),
    "ips_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
    "ips_plan_stage_time": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _i64p]),
    "ips_plan_reset_stage_times": (ctypes.c_int, [_vp]),
    "ips_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ips_last_error_detail": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
}

_lock = threading.Lock()
_lib = None


class IpsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, detail))


def library_path() -> str:
    return LIB_PATH


def lib():
    """Load libipoisson.so once; raise if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libipoisson.so is not built (run python -m paper_2108_11871_amd.build)"
                )
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def detail() -> str:
    buf = ctypes.create_string_buffer(1024)
    lib().ips_last_error_detail(buf, len(buf))
    return buf.value.decode(errors="replace")


def check(status: int):
    if status != IPS_OK:
        raise IpsError(status, detail())
    return status


def i64_array(vals):
    arr = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def f64_array(vals):
    return (ctypes.c_double * len(vals))(*[float(v) for v in vals])
