"""Host-side checks of the C ABI library: it loads without a GPU, exports
every entry point include/tenoaa.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

from paper_2109_14340_amd import tenoaa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "tenoaa.h")).read()
    return sorted(set(re.findall(r"\b(tenoaa_[a-z_]+)\s*\(", src)))


def test_library_exports_header_symbols():
    if not os.path.exists(tenoaa.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(tenoaa.LIB_PATH)
    syms = declared_symbols()
    assert {"tenoaa_rhs", "tenoaa_step", "tenoaa_workspace_bytes"} <= set(syms)
    for name in syms:
        assert hasattr(lib, name), name
    assert sorted(tenoaa.EXPORTS) == sorted(s for s in syms if s in tenoaa.EXPORTS)


def _lib():
    if not os.path.exists(tenoaa.LIB_PATH):
        pytest.skip("library not built")
    return tenoaa.load()


def test_workspace_sizes():
    L = _lib()
    g = tenoaa.make_grid((64, 32, 16))
    s = tenoaa.make_scheme(10)
    rhs = L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 0)
    step = L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 1)
    ncell = 64 * 32 * 16
    assert rhs >= 3 * 5 * ncell * 8
    assert step >= rhs + 5 * ncell * 8
    assert rhs % 256 == 0 and step % 256 == 0


@pytest.mark.parametrize("field,value", [("order", 9), ("splitting", 2), ("positivity", 3)])
def test_bad_scheme_rejected(field, value):
    L = _lib()
    g = tenoaa.make_grid((64,))
    s = tenoaa.make_scheme(10)
    setattr(s, field, value)
    assert L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 0) == 0
    rc = L.tenoaa_rhs(ctypes.byref(g), ctypes.byref(s), 1.4, ctypes.c_void_p(256), ctypes.c_void_p(512), 0.0,
                      None, ctypes.c_void_p(1024), 1 << 30, None)
    assert rc == -1


def test_bad_grid_rejected():
    L = _lib()
    s = tenoaa.make_scheme(10)
    bad = [tenoaa.make_grid((4,)),  # n < G
           tenoaa.make_grid((16, 16), bc_lo=[0, 1], bc_hi=[1, 1]),  # half periodic
           tenoaa.make_grid((16,), dx=[0.0])]
    g = tenoaa.make_grid((16, 16))
    g.n[2] = 3  # unused dimension must be 1
    bad.append(g)
    for g in bad:
        assert L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 0) == 0


def test_bad_call_arguments_rejected():
    L = _lib()
    g = tenoaa.make_grid((64,))
    s = tenoaa.make_scheme(8)
    need = L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 1)
    vp = ctypes.c_void_p
    # gamma <= 1
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.0, 0.4, vp(256), vp(512), vp(1024), need, None) == -1
    # cfl out of range; limiter with cfl > 0.5
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.4, 1.5, vp(256), vp(512), vp(1024), need, None) == -1
    s.positivity = 1
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.4, 0.6, vp(256), vp(512), vp(1024), need, None) == -1
    s.positivity = 0
    # unaligned or small workspace
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.4, 0.4, vp(256), vp(512), vp(1000), need, None) == -1
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.4, 0.4, vp(256), vp(512), vp(1024), need - 8, None) == -5
    # null state, aliased rhs output
    assert L.tenoaa_step(ctypes.byref(g), ctypes.byref(s), 1.4, 0.4, None, vp(512), vp(1024), need, None) == -1
    need_r = L.tenoaa_workspace_bytes(ctypes.byref(g), ctypes.byref(s), 0)
    assert L.tenoaa_rhs(ctypes.byref(g), ctypes.byref(s), 1.4, vp(256), vp(256), 0.0, None, vp(1024), need_r,
                        None) == -1
