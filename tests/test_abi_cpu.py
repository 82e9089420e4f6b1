"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/fsei.h, and plan creation validates its
arguments before anything touches a device."""
import ctypes
import os

import numpy as np
import pytest

from paper_2103_15187_amd import fsei
from paper_2103_15187_amd import workloads as W

pytestmark = pytest.mark.skipif(not os.path.exists(fsei.LIB_PATH), reason="libfsei.so not built")

OK, ERR_ARG, ERR_SIZE, ERR_GRID, ERR_WORKSPACE = 0, -1, -2, -3, -4


def create(nx, ny, nz, bc=(1, 1), dx=0.1, dy=0.1, zc=None):
    L = fsei.lib()
    if zc is None:
        zc = np.linspace(0.0, 1.0, nz + 1)
    zc = np.ascontiguousarray(zc, dtype=np.float64)
    h = ctypes.c_void_p()
    st = L.fsei_poisson_plan_create(nx, ny, nz, (ctypes.c_int * 2)(*bc), dx, dy,
                                    zc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h))
    return st, h


def test_exports_every_declared_function():
    names = fsei.header_functions()
    assert "fsei_poisson_plan_create" in names and "fsei_project_backward" in names
    L = ctypes.CDLL(fsei.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings():
    L = fsei.lib()
    for s in range(-7, 1):
        assert L.fsei_status_string(s).startswith(b"FSEI_")


@pytest.mark.parametrize("n", [1, 5, 7, 10, 4096, 0, -2])
def test_rejects_unsupported_xy_sizes(n):
    st, h = create(n, 8, 8)
    assert st == ERR_SIZE and not h.value


@pytest.mark.parametrize("nz", [1, 0, 2049])
def test_rejects_unsupported_nz(nz):
    zc = np.linspace(0, 1, max(nz, 1) + 1)
    st, h = create(8, 8, nz, zc=zc)
    assert st == ERR_SIZE


def test_rejects_bad_grids():
    zc = np.linspace(0, 1, 9)
    zc[4] = zc[3]
    assert create(8, 8, 8, zc=zc)[0] == ERR_GRID
    zc = np.linspace(0, 1, 9)[::-1].copy()
    assert create(8, 8, 8, zc=zc)[0] == ERR_GRID
    zc = np.linspace(0, 1, 9)
    zc[2] = np.nan
    assert create(8, 8, 8, zc=zc)[0] == ERR_GRID
    assert create(8, 8, 8, dx=0.0)[0] == ERR_GRID
    assert create(8, 8, 8, dy=-1.0)[0] == ERR_GRID
    assert create(8, 8, 8, bc=(2, 1))[0] == ERR_ARG


def test_plan_lifecycle_and_workspace_size_host_only():
    L = fsei.lib()
    for n in (2, 3, 6, 12, 64, 96, 512, 768, 2048):
        st, h = create(n, 8, 8)
        assert st == OK, n
        L.fsei_poisson_plan_destroy(h)
    spec = W.CONFIGS["C3"]
    st, h = create(spec.nx, spec.ny, spec.nz, (spec.bcx, spec.bcy), spec.dx, spec.dy, spec.zc())
    assert st == OK
    sz = ctypes.c_size_t()
    assert L.fsei_plan_workspace_size(h, ctypes.byref(sz)) == OK
    n = spec.ncells
    assert n * 8 <= sz.value < n * 8 + (64 << 20)          # FP64: one field + tables
    assert L.fsei_plan_set_precision(h, fsei.PREC_FP32_REFINE, 1e-10, 4) == OK
    assert L.fsei_plan_workspace_size(h, ctypes.byref(sz)) == OK
    assert n * 24 <= sz.value < n * 24 + (64 << 20)        # f (8) + FP32 work (4) + p (8) + FP32 p (4)
    assert L.fsei_plan_set_precision(h, 7, 1e-10, 4) == ERR_ARG
    assert L.fsei_plan_set_precision(h, 0, -1.0, 4) == ERR_ARG
    assert L.fsei_plan_set_precision(h, 0, 1e-10, 65) == ERR_ARG
    # no workspace set: every compute entry point refuses before launching
    d = ctypes.c_void_p(0x1000)
    assert L.fsei_project(h, d, d, d, d, 1.0, None) == ERR_WORKSPACE
    assert L.fsei_poisson_solve(h, d, d, None) == ERR_WORKSPACE
    assert L.fsei_project_backward(h, d, d, d, None, 1.0) == ERR_WORKSPACE
    assert L.fsei_viscous_solve(h, 0, d, 1e-3) == ERR_WORKSPACE
    L.fsei_poisson_plan_destroy(h)
    L.fsei_poisson_plan_destroy(None)


def test_null_arguments():
    L = fsei.lib()
    assert L.fsei_poisson_plan_create(8, 8, 8, None, 0.1, 0.1, None, None) == ERR_ARG
    assert L.fsei_plan_workspace_size(None, None) == ERR_ARG
    assert L.fsei_project(None, None, None, None, None, 1.0, None) == ERR_ARG
    assert L.fsei_viscous_solve(None, 0, None, 1.0) == ERR_ARG
