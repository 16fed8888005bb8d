"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/emu.h declares, and rejects invalid arguments with LAPACK-style codes
before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2509_23565_amd as emu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "emu.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*|int|size_t)\s*(emu_\w+)\s*\(",
                                 text, re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("emu_dgemm", "emu_dgetrf", "emu_dgetrs"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = emu.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert emu.emu_version() >= 100


def _p(v=0x1000):
    return ctypes.c_void_p(v)   # never dereferenced: argument checks come first


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 7), -1),
    ((4, -1, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 7), -2),
    ((4, 4, -1, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 7), -3),
    ((4, 4, 4, 1.0, None, 4, _p(), 4, 0.0, _p(), 4, 7), -5),
    ((4, 4, 4, 1.0, _p(), 3, _p(), 4, 0.0, _p(), 4, 7), -6),
    ((4, 4, 4, 1.0, _p(), 4, None, 4, 0.0, _p(), 4, 7), -7),
    ((4, 4, 5, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 7), -8),
    ((4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, None, 4, 7), -10),
    ((4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 3, 7), -11),
    ((4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 0), -12),
    ((4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 17), -12),
])
def test_dgemm_argument_errors(args, code):
    assert emu.emu_dgemm(*args) == code
    assert "argument" in emu.emu_last_error()
    # the entry point that allocates nothing checks its arguments the same way
    assert emu.emu_dgemm_noalloc(*args) == code
    assert "argument" in emu.emu_last_error()


def test_dgemm_unsupported_slice_count():
    # 1..16 slices are accepted: with m = 0 the call returns 0 after its
    # argument and support checks, before any device work (the dummy
    # pointers must never reach a kernel); all-pairs thresholds stop at s = 5
    for s in (10, 12, 16):
        assert emu.emu_dgemm(0, 4, 4, 1.0, _p(), 1, _p(), 4, 0.0, _p(), 1, s) == 0
    assert emu.emu_dgemm(0, 4, 4, 1.0, _p(), 1, _p(), 4, 0.0, _p(), 1, 17) == -12
    assert emu.emu_dgemm_t(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 7, 14) == 1003
    assert emu.emu_dgemm_t(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 3, 7) == -13


def test_lu_argument_errors():
    assert emu.emu_dgetrf(-1, 4, _p(), 4, _p(), _p(), 64, 7) == -1
    assert emu.emu_dgetrf(4, 4, _p(), 3, _p(), _p(), 64, 7) == -4
    assert emu.emu_dgetrf(4, 4, _p(), 4, None, _p(), 64, 7) == -5
    assert emu.emu_dgetrf(4, 4, _p(), 4, _p(), None, 64, 7) == -6
    assert emu.emu_dgetrf(4, 4, _p(), 4, _p(), _p(), emu.EMU_MAX_NB + 1, 7) == -7
    assert emu.emu_dgetrf(4, 4, _p(), 4, _p(), _p(), 64, 0) == -8
    assert emu.emu_dgetrf(4, 4, _p(), 4, _p(), _p(), 64, 17) == -8
    assert emu.emu_dgetrs(4, 1, _p(), 3, _p(), _p(), 4) == -4
    assert emu.emu_dgetrs(4, -1, _p(), 4, _p(), _p(), 4) == -2
    assert emu.emu_dgetrs(4, 1, _p(), 4, _p(), _p(), 2) == -7
    assert emu.emu_status(None) == -1
    for key in ("lu_pivot", "lu_update", "gemm_map", "leaf_cooperative", "leaf_one_xcd"):
        assert emu.emu_set_param(key.encode(), 2) == -2


def test_workspace_calls_argument_codes_and_sizes():
    assert emu.emu_set_workspace(None, 4096) == -1
    assert emu.emu_workspace_bytes(-1, 4, 4, 7) == 0
    assert emu.emu_workspace_bytes(4, 4, 4, 0) == 0
    assert emu.emu_workspace_bytes(4, 4, 4, emu.EMU_MAX_SLICES + 1) == 0
    assert emu.emu_workspace_bytes(0, 4, 4, 7) == 0
    # digit planes: s planes of lines padded to 128 and K to 32, 1 byte each
    small = emu.emu_workspace_bytes(100, 100, 100, 3)
    assert small >= 2 * 3 * 128 * 128
    assert emu.emu_workspace_bytes(100, 100, 100, 7) > small
    assert emu.emu_getrf_workspace_bytes(4, 4, emu.EMU_MAX_NB + 1, 7) == 0
    assert emu.emu_getrf_workspace_bytes(4000, 4000, 2048, 7) > 0
    assert emu.emu_getrf_workspace_bytes(1000, 1000, 128, 7) > 0
    assert emu.emu_getrs_workspace_bytes(-1, 1) == 0
    assert emu.emu_getrs_workspace_bytes(1000, 2) >= 1000 * 2 * 8


def test_batched_refinement_argument_codes():
    n = (ctypes.c_int * 1)(8)
    r = (ctypes.c_int * 1)(1)
    ld = (ctypes.c_int * 1)(8)
    P = (ctypes.c_void_p * 1)(0x1000)
    it = (ctypes.c_int * 1)()
    be = (ctypes.c_double * 1)()
    sf = (ctypes.c_int * 1)()
    inf = (ctypes.c_int * 1)()
    f = emu.emu_dgesv_batched_ir
    assert f(-1, n, r, P, ld, P, ld, P, ld, 32, 3, 1e-15, 10, it, be, sf, inf) == -1
    assert f(1, n, r, P, ld, P, ld, P, ld, 33, 3, 1e-15, 10, it, be, sf, inf) == -10
    assert f(1, n, r, P, ld, P, ld, P, ld, 32, 10, 1e-15, 10, it, be, sf, inf) == -11
    assert f(1, n, r, P, ld, P, ld, P, ld, 32, 3, 0.0, 10, it, be, sf, inf) == -12
    assert f(1, n, r, P, ld, P, ld, P, ld, 32, 3, 1e-15, -1, it, be, sf, inf) == -13
    assert f(1, n, r, P, ld, P, ld, P, ld, 32, 3, 1e-15, 10, None, be, sf, inf) == -14
    big = (ctypes.c_int * 1)(2000)
    assert f(1, big, r, P, big, P, big, P, big, 32, 3, 1e-15, 10, it, be, sf, inf) == 1003
    assert f(0, None, None, None, None, None, None, None, None, 32, 3, 1e-15, 10, None, None,
             None, None) == 0


def test_batched_solve_argument_codes():
    n = (ctypes.c_int * 1)(8)
    r = (ctypes.c_int * 1)(1)
    ld = (ctypes.c_int * 1)(8)
    short = (ctypes.c_int * 1)(7)
    P = (ctypes.c_void_p * 1)(0x1000)
    Z = (ctypes.c_void_p * 1)(0)
    f = emu.emu_dgetrs_batched
    assert f(-1, n, r, P, ld, P, P, ld) == -1
    assert f(0, None, None, None, None, None, None, None) == 0
    assert f(1, None, r, P, ld, P, P, ld) == -2
    assert f(1, n, None, P, ld, P, P, ld) == -3
    assert f(1, n, r, Z, ld, P, P, ld) == -4
    assert f(1, n, r, P, short, P, P, ld) == -5
    assert f(1, n, r, P, ld, Z, P, ld) == -6
    assert f(1, n, r, P, ld, P, Z, ld) == -7
    assert f(1, n, r, P, ld, P, P, short) == -8
    big = (ctypes.c_int * 1)(1025)
    assert f(1, big, r, P, big, P, P, big) == 1003
    many = (ctypes.c_int * 1)(9)
    assert f(1, n, many, P, ld, P, P, ld) == 1003


def test_getrf_autotune_argument_codes():
    f = emu.emu_autotune_getrf
    nb, ms = ctypes.c_int(0), ctypes.c_double(0.0)
    bn, bm = ctypes.byref(nb), ctypes.byref(ms)
    assert f(0, 4, _p(), 4, 3, None, 0, bn, bm) == -1
    assert f(4, 0, _p(), 4, 3, None, 0, bn, bm) == -2
    assert f(4, 4, None, 4, 3, None, 0, bn, bm) == -3
    assert f(4, 4, _p(), 3, 3, None, 0, bn, bm) == -4
    assert f(4, 4, _p(), 4, 0, None, 0, bn, bm) == -5
    assert f(4, 4, _p(), 4, 17, None, 0, bn, bm) == -5
    assert f(4, 4, _p(), 4, 3, None, 2, bn, bm) == -6
    assert f(4, 4, _p(), 4, 3, (ctypes.c_int * 1)(4096), 1, bn, bm) == -6
    assert f(4, 4, _p(), 4, 3, (ctypes.c_int * 1)(0), 1, bn, bm) == -6
    assert f(4, 4, _p(), 4, 3, None, -1, bn, bm) == -7
    assert f(4, 4, _p(), 4, 3, None, 0, None, bm) == -8
    assert f(4, 4, _p(), 4, 3, None, 0, bn, None) == -9


def test_unequal_splits_argument_codes():
    f = emu.emu_dgemm_ab
    assert f(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 9, 0) == -13
    assert f(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 5, 6) == -13
    assert f(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 0, 1) == -12
    assert f(4, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 12, 3) == 1003
    assert f(-1, 4, 4, 1.0, _p(), 4, _p(), 4, 0.0, _p(), 4, 9, 3) == -1
