"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/cta.h declares, and
reject invalid arguments with a status code before touching the device.
"""
import ctypes
import os

import pytest

import paper_1001_5460_amd as cta

LIB = cta.library_path()
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcta.so not built")


def test_exports_every_declared_symbol():
    lib = cta.load_library()
    syms = cta.exported_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in cta.cta_version()


def test_op_create_rejects_bad_order():
    lib = cta.load_library()
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 1)(4)
    st = lib.cta_op_create(ctypes.byref(h), 1, n, n, None, None, None, 0.0, None)
    assert st == -1 and "order" in cta.cta_last_error()
    st = lib.cta_op_create(None, 3, n, n, None, None, None, 0.0, None)
    assert st == -1


def test_op_create_rejects_large_extent():
    lib = cta.load_library()
    h = ctypes.c_void_p()
    n = (ctypes.c_int64 * 3)(4, 300, 4)
    A = (ctypes.c_void_p * 3)(1, 1, 1)
    st = lib.cta_op_create(ctypes.byref(h), 3, n, n, A, None, None, 0.0, None)
    assert st == -2 and "extents" in cta.cta_last_error()


def test_ttm_workspace_planning():
    # rectangular chain: workspace holds padded factors plus two buffers of
    # the largest intermediate (the planner's order)
    b = cta.cta_ttm_workspace_bytes([192, 192, 144, 36], [(192, 128), (192, 128), (144, 96), (36, 24)],
                                    trans=(0, 1, 2, 3), compute="f64")
    assert b >= 2 * 192 * 192 * 144 * 36 * 8
    assert cta.cta_ttm_workspace_bytes([4, 5], [(3, 6), None]) == 0   # shape mismatch


def test_ttm_rejects_shape_mismatch_without_device():
    lib = cta.load_library()
    dims = (ctypes.c_int64 * 2)(4, 5)
    rows = (ctypes.c_int64 * 2)(3, 0)
    cols = (ctypes.c_int64 * 2)(6, 0)
    st = lib.cta_ttm(2, dims, None, 1, 1, 0, None, rows, cols, 1, 1, None, 1, None, 0, None)
    assert st == -2


def test_cg_solve_rejects_null():
    lib = cta.load_library()
    st = lib.cta_cg_solve(None, None, None, 1, None, None, None)
    assert st == -1


def test_default_options():
    o = cta.cta_cg_opts_default()
    assert o["rtol"] == 1e-6 and o["check_every"] == 16 and o["precision"] == cta.PREC_F32


def test_option_struct_matches_header():
    """The binding's cta_cg_opts mirror has the C layout: the library's
    default writer fills every field, including the last one."""
    import ctypes
    from paper_1001_5460_amd import _lib
    o = _lib._CgOpts()
    o.precond = 7
    cta.load_library().cta_cg_opts_default(ctypes.byref(o))
    assert o.precond == 0 and o.max_refine == 30
    assert ctypes.sizeof(_lib._CgOpts) == 56
