"""Host-side checks of the C ABI (no GPU): the library loads, exports every symbol that
include/ed.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1802_10052_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ed.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ed_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    syms = declared_symbols()
    assert "ed_apply_H" in syms and len(syms) >= 7
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def _desc(L=4, d=2, n_site=1, n_bond=1, null_ops=False):
    so = np.zeros((n_site, 2, 2), np.complex128)
    sc = np.ones((n_site, L))
    bo = np.zeros((n_bond, 4, 4), np.complex128)
    bc = np.ones((n_bond, max(L - 1, 1)))
    keep = (so, sc, bo, bc)
    d_ = _lib.ModelDescC(L, d, n_site, None if null_ops else so.ctypes.data, sc.ctypes.data,
                         n_bond, bo.ctypes.data, bc.ctypes.data)
    return d_, keep


def test_model_create_argument_errors():
    lib = _lib.lib()
    h = C.c_void_p()
    assert lib.ed_model_create(None, C.byref(h)) == -1
    d, keep = _desc(d=3)
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -2
    d, keep = _desc(L=31)
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -2
    d, keep = _desc(L=1)
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -2
    d, keep = _desc(null_ops=True)
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -1
    assert b"null" in lib.ed_last_error()
    d, keep = _desc()
    keep[1][0, 0] = np.nan
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -8


def test_apply_rejects_null_arguments():
    lib = _lib.lib()
    assert lib.ed_apply_H(None, None, None, None) == -1
    n = C.c_int(-5)
    assert lib.ed_trotter_passes(None, 4, C.byref(n)) == -1 and n.value == -5


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be visible")
def test_model_create_without_device_reports_nodevice():
    lib = _lib.lib()
    d, keep = _desc()
    h = C.c_void_p()
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -3


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be visible")
def test_pass_plans_valid_for_every_length():
    """Model creation checks its H psi pass plan (every site and bond in exactly one pass) before
    looking for a device: on a CPU-only host every L must get as far as ED_ERR_NODEVICE."""
    lib = _lib.lib()
    for L in range(2, 31):
        for flip_bonds in (True, False):
            d, keep = _desc(L=L, n_site=2, n_bond=2)
            keep[0][:] = np.array([[0, 1], [1, 0]])   # off-diagonal sites
            keep[2][:] = 0.0
            keep[2][:, 0, 0] = 1.0                     # diagonal bond part (zz-like)
            if flip_bonds:
                keep[2][:, 0, 3] = 1.0                 # double-flip bonds: passes must overlap
            h = C.c_void_p()
            assert lib.ed_model_create(C.byref(d), C.byref(h)) == -3, (L, flip_bonds, lib.ed_last_error())


@pytest.mark.skipif(os.environ.get("HIP_VISIBLE_DEVICES") is None and os.path.exists("/dev/kfd"),
                    reason="a GPU may be visible")
def test_long_range_rule_validation():
    """InfiniteFunc rules are folded and checked before the device is looked for: diagonal
    operators reach ED_ERR_NODEVICE on a CPU-only host, off-diagonal ones ED_ERR_UNSUPPORTED, null
    arrays with n_inf > 0 ED_ERR_ARG."""
    lib = _lib.lib()
    L = 14
    d, keep = _desc(L=L, n_site=1, n_bond=1)
    keep[0][:] = np.array([[0, 1], [1, 0]])
    o1 = np.array([[[1, 0], [0, -1]]], np.complex128)
    o2 = np.array([[[0.5, 0], [0, 2j]]], np.complex128)
    ic = np.ones((1, L))
    fr = 1.0 / np.arange(1, L, dtype=np.float64).reshape(1, L - 1) ** 1.5
    d.n_inf, d.inf_op, d.inf_op2, d.inf_coef, d.inf_f = 1, o1.ctypes.data, o2.ctypes.data, ic.ctypes.data, fr.ctypes.data
    h = C.c_void_p()
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -3, lib.ed_last_error()
    hop = np.array([[[0, 1], [0, 0]]], np.complex128)
    d.inf_op2 = hop.ctypes.data
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -2
    assert b"diagonal" in lib.ed_last_error()
    d.inf_op2 = None
    assert lib.ed_model_create(C.byref(d), C.byref(h)) == -1


def test_liouville_create_validation():
    """ed_liouville_create checks its arguments before touching a device."""
    lib = C.CDLL(_lib.LIB_PATH)
    lib.ed_liouville_create.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    sm = np.array([[0, 0], [1, 0]], np.complex128)

    def call(L, rates, n_jump=1, jump=sm):
        d, keep = _desc(L=L)
        r = np.ascontiguousarray(rates, np.float64)
        h = C.c_void_p()
        return lib.ed_liouville_create(C.byref(d), n_jump, jump.ctypes.data if jump is not None else None,
                                       r.ctypes.data, C.byref(h))
    assert call(16, np.full((1, 16), 0.1)) == -2          # the superket would have 32 bits
    assert call(4, np.array([[0.1, -0.1, 0.1, 0.1]])) == -1
    assert call(4, np.full((1, 4), np.nan)) == -1
    assert call(4, np.full((1, 4), 0.1), jump=None) == -1
    assert call(4, np.full((1, 4), 0.1), n_jump=-1) == -1
    assert call(4, np.full((1, 4), 0.1)) in (0, -3)       # valid: fails only for want of a device
