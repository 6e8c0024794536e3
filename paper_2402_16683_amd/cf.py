"""Binding of the correlated-field model and its Poisson Fisher metric (include/icr_cf.h).

Argument marshalling only: every step runs in the library's kernels. Fields are FP32
device tensors of shape (n, n).
"""

from __future__ import annotations

import ctypes

from .icr import _check, _stream_handle, load_library

_sigs_done = False


def _lib():
    global _sigs_done
    lib = load_library()
    if not _sigs_done:
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        sigs = {
            "icr_cf_create": [i32, d, d, d, d, d, vp, ctypes.POINTER(vp)],
            "icr_cf_workspace_bytes": [vp, ctypes.POINTER(i64)],
            "icr_cf_copy_amplitude": [vp, vp],
            "icr_cf_transform": [vp, vp, vp, vp, vp],
            "icr_cf_rate": [vp, vp, vp, vp, vp],
            "icr_cf_metric_apply": [vp, vp, vp, vp, vp, vp],
            "icr_cf_destroy": [vp],
        }
        for name, args in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _sigs_done = True
    return lib


class CorrelatedField:
    """An n x n correlated field with amplitude a (1 + (|k| l)^2)^(-slope/4), zero mode a0,
    and a Poisson rate exp(offset_mean + T(A xi)); owns the device workspace."""

    def __init__(self, n: int, amplitude: float = 1.0, zero_mode: float = 0.1, length: float = 0.05,
                 slope: float = 3.0, offset_mean: float = 2.0, stream=None):
        import torch
        self.n = n
        self.params = dict(amplitude=amplitude, zero_mode=zero_mode, length=length, slope=slope,
                           offset_mean=offset_mean)
        h = ctypes.c_void_p()
        _check(_lib().icr_cf_create(n, amplitude, zero_mode, length, slope, offset_mean, _stream_handle(stream),
                                    ctypes.byref(h)))
        self.handle = h
        nb = ctypes.c_int64()
        _check(_lib().icr_cf_workspace_bytes(self.handle, ctypes.byref(nb)))
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device="cuda")

    def _field(self, t, name):
        import torch
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.numel() == self.n * self.n):
            raise ValueError(f"{name} must be a contiguous float32 device tensor of {self.n}x{self.n}")
        return ctypes.c_void_p(t.data_ptr())

    def _new(self):
        import torch
        return torch.empty((self.n, self.n), dtype=torch.float32, device="cuda")

    def amplitude(self):
        import numpy as np
        out = np.empty((self.n, self.n), dtype=np.float32)
        _check(_lib().icr_cf_copy_amplitude(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def transform(self, x, out=None, stream=None):
        out = self._new() if out is None else out
        _check(_lib().icr_cf_transform(self.handle, self._field(x, "x"), self._field(out, "out"),
                                       ctypes.c_void_p(self.workspace.data_ptr()), _stream_handle(stream)))
        return out

    def rate(self, position, out=None, stream=None):
        """lambda = exp(offset_mean + T(A position)): builds M_p at the position."""
        out = self._new() if out is None else out
        _check(_lib().icr_cf_rate(self.handle, self._field(position, "position"), self._field(out, "lambda"),
                                  ctypes.c_void_p(self.workspace.data_ptr()), _stream_handle(stream)))
        return out

    def metric_apply(self, lam, v, out=None, stream=None):
        """M_p v = v + A T(lambda T(A v))."""
        out = self._new() if out is None else out
        _check(_lib().icr_cf_metric_apply(self.handle, self._field(lam, "lambda"), self._field(v, "v"),
                                          self._field(out, "out"), ctypes.c_void_p(self.workspace.data_ptr()),
                                          _stream_handle(stream)))
        return out

    def __del__(self):
        try:
            if self.handle:
                _lib().icr_cf_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
