"""Host-side checks of the C ABI that run without a GPU: the library loads,
exports every entry point declared in include/lmfmm.h, and rejects bad
arguments with status codes before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1902_08250_amd import lmfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lmfmm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lmfmm_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for name in ("lmfmm_create", "lmfmm_apply", "lmfmm_apply_adjoint", "lmfmm_destroy"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = lmfmm.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(lmfmm.EXPORTS) <= set(declared_symbols())


def _create(k, d, order, tol):
    L = lmfmm.lib()
    arr = (ctypes.c_double * 6)(*k)
    h = ctypes.c_void_p()
    rc = L.lmfmm_create(arr, d, order, tol, ctypes.byref(h))
    return rc, h


K_OK = (10, 0.01, 20, 0.01, 15, 0.01)


@pytest.mark.parametrize("k,d,order,tol", [
    ((10, -0.1, 20, 0.01, 15, 0.01), 1.0, 16, 1e-6),   # Im k < 0
    ((0, 0.01, 20, 0.01, 15, 0.01), 1.0, 16, 1e-6),    # Re k = 0
    (K_OK, 0.0, 16, 1e-6),                              # d = 0
    (K_OK, 1.0, 0, 1e-6),                               # order < 1
    (K_OK, 1.0, 300, 1e-6),                             # order too large
    (K_OK, 1.0, 16, 0.0),                               # tol = 0
    (K_OK, 1.0, 16, 1.5),                               # tol >= 1
    ((float("nan"), 0, 20, 0, 15, 0), 1.0, 16, 1e-6),  # non-finite
])
def test_create_rejects_bad_arguments(k, d, order, tol):
    rc, h = _create(k, d, order, tol)
    assert rc == lmfmm.EINVAL
    assert not h.value
    assert lmfmm.lib().lmfmm_last_error()


def test_null_arguments():
    L = lmfmm.lib()
    assert L.lmfmm_create(None, 1.0, 16, 1e-6, None) == lmfmm.EINVAL
    assert L.lmfmm_destroy(None) == lmfmm.EINVAL
    assert L.lmfmm_apply(None, 0, None, None, 0, None, None, 1, 0, None) == lmfmm.EINVAL
    assert L.lmfmm_apply_adjoint(None, 0, None, 0, None, None, None, 1, 0, None) == lmfmm.EINVAL
    assert L.lmfmm_get_stats(None, None) == lmfmm.EINVAL
    assert L.lmfmm_set_option(None, b"levels", b"3") == lmfmm.EINVAL


def test_status_strings():
    L = lmfmm.lib()
    for s in (0, -1, -2, -3, -4, -5, -6):
        assert L.lmfmm_status_string(s)
