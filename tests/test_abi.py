"""The C-ABI library loads, exports every entry point include/mpde.h
declares, and rejects invalid arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

from paper_2502_18377_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mpde.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(mpde_[a-z0-9_]+)\s*\(", src))


def test_exports_match_header():
    lib = N.load()
    declared = _declared()
    assert declared == set(N.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_default_options():
    lib = N.load()
    o = N.Options()
    assert lib.mpde_default_options(ctypes.byref(o)) == 0
    assert o.tol == 1e-6 and o.nu == 2 and o.max_inner == 200 and o.coarse_min == 8
    assert lib.mpde_default_options(None) == N.MPDE_ERR_INVALID_ARG


def _desc(**kw):
    d = N.Desc()
    shape = (ctypes.c_int32 * 2)(8, 8)
    step = (ctypes.c_double * 2)(0.1, 0.1)
    d.dtype, d.ndim, d.batch = N.MPDE_F32, 2, 1
    d.shape = ctypes.cast(shape, ctypes.POINTER(ctypes.c_int32))
    d.step = ctypes.cast(step, ctypes.POINTER(ctypes.c_double))
    d.bc_lo[0], d.bc_lo[1], d.bc_hi[1] = N.MPDE_BC_DIRICHLET, N.MPDE_BC_DIRICHLET, N.MPDE_BC_DIRICHLET
    d.mset = 0b11011
    d.coeff = d.rhs = d.bc_values = 0x1000          # never dereferenced: validation fails first
    for k, v in kw.items():
        setattr(d, k, v)
    d._keep = (shape, step)
    return d


@pytest.mark.parametrize("field,value", [("dtype", 7), ("ndim", 4), ("batch", 0), ("mset", 0),
                                          ("mset", 1 << 5), ("coeff", None)])
def test_invalid_arguments_rejected(field, value):
    lib = N.load()
    h = ctypes.c_void_p()
    d = _desc(**{field: value})
    assert lib.mpde_build(ctypes.byref(d), ctypes.byref(h)) in (N.MPDE_ERR_INVALID_ARG, N.MPDE_ERR_UNSUPPORTED)
    assert not h.value
    assert lib.mpde_last_error()


def test_small_axis_and_bad_periodic_rejected():
    lib = N.load()
    h = ctypes.c_void_p()
    d = _desc()
    d.shape[1] = 4
    assert lib.mpde_build(ctypes.byref(d), ctypes.byref(h)) == N.MPDE_ERR_INVALID_ARG
    d = _desc()
    d.bc_lo[1], d.bc_hi[1] = N.MPDE_BC_PERIODIC, N.MPDE_BC_DIRICHLET
    assert lib.mpde_build(ctypes.byref(d), ctypes.byref(h)) == N.MPDE_ERR_INVALID_ARG
    assert b"periodic" in lib.mpde_last_error()


def test_null_handles():
    lib = N.load()
    lib.mpde_free(None)
    assert lib.mpde_solve(None, None, None) == N.MPDE_ERR_INVALID_ARG
    assert lib.mpde_solve_adjoint(None, None, None, None, None, None) == N.MPDE_ERR_INVALID_ARG
    assert lib.mpde_levels(None, 0, None) == 0
    assert lib.mpde_build(None, None) == N.MPDE_ERR_INVALID_ARG


def test_no_device_reported_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = N.load()
    h = ctypes.c_void_p()
    d = _desc()
    assert lib.mpde_build(ctypes.byref(d), ctypes.byref(h)) == N.MPDE_ERR_NO_DEVICE
