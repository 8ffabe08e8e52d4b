"""MI355X-native exact-diagonalisation hot path (Jaschke & Carr, arXiv:1802.10052).

Python face of libed.so: device memory and streams come from torch; the product H psi and all
the methods built on it run in the library's HIP kernels. Names follow the C ABI (include/ed.h).
"""
import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import EdError, call, lib

__all__ = ["Model", "apply_H", "EdError", "lib"]


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _check_state(t, D, name="psi"):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if t.numel() != D or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {D} elements")


class Model:
    """Handle on an immutable rule-set Hamiltonian (site + bond rules).

    desc: any object with L, site_ops (n,2,2), site_coef (n,L), bond_ops (m,4,4),
    bond_coef (m,L-1) (e.g. edinputs.ModelDesc). The handle lives on the current device.
    """

    def __init__(self, desc):
        self.L = int(desc.L)
        self._keep = [np.ascontiguousarray(desc.site_ops, np.complex128),
                      np.ascontiguousarray(desc.site_coef, np.float64),
                      np.ascontiguousarray(desc.bond_ops, np.complex128),
                      np.ascontiguousarray(desc.bond_coef, np.float64)]
        so, sc, bo, bc = self._keep
        d = _lib.ModelDescC(self.L, 2, len(so), so.ctypes.data, sc.ctypes.data,
                            len(bo), bo.ctypes.data, bc.ctypes.data)
        h = C.c_void_p()
        call("ed_model_create", C.byref(d), C.byref(h))
        self._h = h
        self.D = 1 << self.L

    @property
    def handle(self):
        return self._h

    @property
    def passes(self):
        n = C.c_int()
        call("ed_model_passes", self._h, C.byref(n))
        return n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().ed_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_H(model, psi, out=None, stream=None):
    """out = H psi (asynchronous on the current torch stream)."""
    _check_state(psi, model.D)
    if out is None:
        out = torch.empty_like(psi)
    _check_state(out, model.D, "out")
    call("ed_apply_H", model.handle, _dptr(psi), _dptr(out), _stream_ptr(stream))
    return out
