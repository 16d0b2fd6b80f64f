"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every declared entry point, and rejects invalid arguments before touching a
device."""
import ctypes
import os
import re

import pytest

from paper_2108_11871_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ipoisson.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ips_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    syms = declared_symbols()
    for name in ("ips_solve", "ips_plan_create", "ips_execute", "ips_execute_adjoint",
                 "ips_plan_destroy", "ips_batch_create", "ips_batch_execute",
                 "ips_batch_destroy", "ips_status_string", "ips_last_error_detail",
                 "ips_plan_workspace_size"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
        assert name in _lib.SIGNATURES, name


def _create(d, n, h, order=6, precision=0, flags=0):
    L = _lib.lib()
    handle = ctypes.c_void_p()
    rc = L.ips_plan_create(ctypes.byref(handle), d, _lib.i64_array(n), _lib.f64_array(h), order,
                           precision, flags)
    return rc, handle


@pytest.mark.parametrize(
    "args,code",
    [
        ((0, [9], [0.1]), -1),
        ((4, [9, 9, 9, 9], [0.1] * 4), -1),
        ((2, [2, 9], [0.1, 0.1]), -1),
        ((2, [9, 9], [0.0, 0.1]), -1),
        ((2, [9, 9], [float("nan"), 0.1]), -1),
        ((2, [9, 9], [float("inf"), 0.1]), -1),
        ((3, [9, 9, 7], [0.1] * 3), -1),  # order 6 needs n >= 8
        ((2, [9, 4098], [0.1, 0.1]), -2),  # 2D: transforms longer than 8192
        ((3, [9, 9, 1026], [0.1, 0.1, 0.1]), -2),  # 3D: transforms longer than 2048
    ],
)
def test_plan_create_rejects_bad_geometry(args, code):
    rc, handle = _create(*args)
    assert rc == code
    assert not handle.value
    assert _lib.detail()


def test_plan_create_rejects_bad_order_precision_flags():
    assert _create(2, [9, 9], [0.1, 0.1], order=5)[0] == -1
    assert _create(2, [9, 9], [0.1, 0.1], precision=7)[0] == -1
    assert _create(2, [9, 9], [0.1, 0.1], flags=64)[0] == -1
    assert _create(2, [9, 9], [0.1, 0.1], flags=128)[0] == -1  # direct surface sums need screening
    assert _create(2, [9, 9], [0.1, 0.1], flags=256)[0] == -1
    assert _create(2, [9, 9], [0.1, 0.1], precision=1, flags=32)[0] == -2
    assert _create(2, [9, 9], [0.1, 0.1], flags=32 | 2)[0] == -2
    assert _create(3, [9, 6, 9], [0.1, 0.1, 0.1], order=4, flags=32)[0] == -1
    assert _create(1, [9], [0.1], precision=1)[0] == -2


def test_null_arguments_are_rejected():
    L = _lib.lib()
    assert L.ips_plan_create(None, 2, _lib.i64_array([9, 9]), _lib.f64_array([0.1, 0.1]), 6, 0, 0) == -1
    h = ctypes.c_void_p()
    assert L.ips_plan_create(ctypes.byref(h), 2, None, _lib.f64_array([0.1, 0.1]), 6, 0, 0) == -1
    assert L.ips_execute(None, None, None, None) == -1
    assert L.ips_execute_adjoint(None, None, None, None) == -1
    n = ctypes.c_size_t()
    assert L.ips_plan_workspace_size(None, ctypes.byref(n)) == -1
    assert L.ips_plan_table_size(None, ctypes.byref(n)) == -1
    assert L.ips_plan_set_workspace(None, None, 0) == -1
    assert L.ips_live_device_bytes(None) == -1
    assert L.ips_solve_cache_size(None) == -1
    assert L.ips_solve_cache_size(ctypes.byref(n)) == 0 and n.value == 0
    assert L.ips_live_device_bytes(ctypes.byref(n)) == 0 and n.value == 0
    assert L.ips_solve_release_cache() == 0


def test_solve_ex_rejects_bad_precision_before_the_device():
    L = _lib.lib()
    n = _lib.i64_array([9, 9, 9])
    h = _lib.f64_array([0.1] * 3)
    assert L.ips_solve_ex(3, n, h, None, 6, 9, None) == -1
    assert L.ips_solve_ex(1, _lib.i64_array([9]), _lib.f64_array([0.1]), None, 6, 1, None) == -2
    assert L.ips_solve_ex(3, n, h, None, 6, 0, None) == -1  # NULL arrays
    assert L.ips_solve(2, _lib.i64_array([9, 9]), _lib.f64_array([0.1, 0.1]), None, 6, None) == -1
    n = ctypes.c_size_t()
    assert L.ips_plan_workspace_size(None, ctypes.byref(n)) == -1
    assert L.ips_plan_destroy(None) == 0
    assert L.ips_batch_destroy(None) == 0
    assert L.ips_last_error_detail(None, 8) == -1


def test_status_strings():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -5, 42):
        s = L.ips_status_string(code)
        assert isinstance(s, bytes) and s


def test_last_error_detail_truncates():
    L = _lib.lib()
    _create(0, [9], [0.1])
    buf = ctypes.create_string_buffer(5)
    assert L.ips_last_error_detail(buf, 5) == 0
    assert len(buf.value) == 4


def _smooth235(m):
    for q in (2, 3, 5):
        while m % q == 0:
            m //= q
    return m == 1


@pytest.mark.parametrize("n,margin", [((3,), (0,)), ((257, 257, 257), (8, 8, 8)), ((65, 80), (3, 0)),
                                      ((97, 33, 41), (5, 1, 12)), ((1025,), (7,)), ((11, 12, 13), (0, 0, 0))])
def test_extension_grid(n, margin):
    """ips_extension: every axis gets at least 2 margin nodes more, then the
    smallest count whose panel count has no prime factor above 5; the caller's
    block sits margin nodes plus half the rounding from the low end."""
    L = _lib.lib()
    d = len(n)
    ne = (ctypes.c_int64 * d)()
    off = (ctypes.c_int64 * d)()
    assert L.ips_extension(d, _lib.i64_array(n), _lib.i64_array(margin), ne, off) == 0
    for a in range(d):
        need = n[a] + 2 * margin[a]
        assert ne[a] >= need and _smooth235(ne[a] - 1)
        assert all(not _smooth235(m - 1) for m in range(need, ne[a]))
        assert off[a] == margin[a] + (ne[a] - need) // 2
        assert off[a] >= margin[a] and ne[a] - off[a] - n[a] >= margin[a]


def test_extension_rejects_invalid_arguments():
    """-1 is IPS_E_INVALID_ARG."""
    L = _lib.lib()
    ne = (ctypes.c_int64 * 3)()
    off = (ctypes.c_int64 * 3)()
    assert L.ips_extension(0, _lib.i64_array((5,)), _lib.i64_array((1,)), ne, off) == -1
    assert L.ips_extension(1, _lib.i64_array((2,)), _lib.i64_array((1,)), ne, off) == -1
    assert L.ips_extension(1, _lib.i64_array((9,)), _lib.i64_array((-1,)), ne, off) == -1
    assert L.ips_extension(1, _lib.i64_array((9,)), None, ne, off) == -1
