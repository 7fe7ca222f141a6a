"""Python binding of the double FFT filter (argument marshalling only).

Every step of the filter runs in libsphfilt.so's HIP kernels; this module
checks tensor shapes and dtypes, passes raw device pointers and the current
HIP stream through the C-ABI, and raises on a non-zero status.  PyTorch
provides device memory and streams.

The operator (arXiv:2305.01537, Sec. II.B): theta-filter on lines extended
across the poles, then phi-filter on rings, with cutoffs l_max = max(2, 2 rho L)
and m_max = max(2, 2 rho sin(theta) L).  Its transpose is the phi-pass
followed by the theta-pass; SphFilter uses it as the backward.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import EXP, GAUSS, SHARP, SphfiltError, status_string  # noqa: F401


def _as_int_array(v, n, name):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.int32), (n,)))
    if a.shape != (n,):
        raise ValueError(f"{name} must have {n} entries")
    return a


def _as_double_array(v, n, name):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)))
    if a.shape != (n,):
        raise ValueError(f"{name} must have {n} entries")
    return a


class _Params:
    """Host copies of the per-field / per-shell parameters and their C views."""

    def __init__(self, n_r, n_fields, parity, L, rho, kind, floor_modes):
        self.parity = _as_int_array(parity, n_fields, "parity")
        self.L = _as_double_array(L, n_fields, "L")
        self.rho = None if rho is None else _as_double_array(rho, n_r, "rho")
        self.kind = None if kind is None else _as_int_array(kind, n_fields, "kind")
        self.cut = _lib.Cutoff(
            None if self.rho is None else self.rho.ctypes.data_as(_lib.c_double_p),
            self.L.ctypes.data_as(_lib.c_double_p),
            None if self.kind is None else self.kind.ctypes.data_as(_lib.c_int_p),
            float(floor_modes))

    @property
    def parity_p(self):
        return self.parity.ctypes.data_as(_lib.c_int_p)


def workload_stats(n_r, n_theta, n_phi, n_fields, parity=1, L=3.0, rho=None, kind=None,
                   floor_modes=2.0) -> dict:
    """Active lines and algorithmic HBM bytes of a filter call (host only)."""
    prm = _Params(n_r, n_fields, parity, L, rho, kind, floor_modes)
    st = _lib.Stats()
    _lib.check("sphfilt_workload_stats",
               _lib.load().sphfilt_workload_stats(n_r, n_theta, n_phi, n_fields, prm.parity_p,
                                                  ctypes.byref(prm.cut), ctypes.byref(st)))
    return st.as_dict()


def _stream_handle(x, stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(x.device)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A filter plan for n_fields FP64 fields on an n_r x n_theta x n_phi grid.

    parity: +1/-1 per field (axis parity); L: cutoff scale per field;
    rho: r/dr_min per shell (None: i + 1/2); kind: EXP/GAUSS/SHARP per field
    (None: EXP); floor_modes: the cutoff floor (2 in the paper).
    The plan's tables live on the current HIP device.
    """

    def __init__(self, n_r: int, n_theta: int, n_phi: int, n_fields: int, parity=1, L=3.0,
                 rho=None, kind=None, floor_modes: float = 2.0):
        self.shape = (int(n_fields), int(n_r), int(n_theta), int(n_phi))
        self._prm = _Params(n_r, n_fields, parity, L, rho, kind, floor_modes)
        h = ctypes.c_void_p()
        lib = _lib.load()
        _lib.check("sphfilt_plan_create",
                   lib.sphfilt_plan_create(ctypes.byref(h), n_r, n_theta, n_phi, n_fields,
                                           self._prm.parity_p, ctypes.byref(self._prm.cut)))
        self._h = h
        self._lib = lib

    # -- lifetime -------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sphfilt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- calls ----------------------------------------------------------
    def _check_tensor(self, x, name):
        import torch
        if not isinstance(x, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if x.dtype != torch.float64:
            raise TypeError(f"{name} must be float64")
        if x.device.type != "cuda":
            raise ValueError(f"{name} must live on a HIP device")
        if tuple(x.shape) != self.shape:
            raise ValueError(f"{name} has shape {tuple(x.shape)}, plan expects {self.shape}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _call(self, fname, x, out, stream):
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_tensor(out, "out")
        rc = getattr(self._lib, fname)(self._h, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _stream_handle(x, stream))
        _lib.check(fname, rc)
        return out

    def apply(self, x, out=None, stream=None):
        """out = Phi(Theta(x)); pass out=x to filter in place."""
        return self._call("sphfilt_apply", x, out, stream)

    def apply_adjoint(self, x, out=None, stream=None):
        """out = Theta(Phi(x)), the transpose of apply."""
        return self._call("sphfilt_apply_adjoint", x, out, stream)

    def apply_theta(self, x, out=None, stream=None):
        return self._call("sphfilt_apply_theta", x, out, stream)

    def apply_phi(self, x, out=None, stream=None):
        return self._call("sphfilt_apply_phi", x, out, stream)

    # -- introspection / tuning ------------------------------------------
    def stats(self) -> dict:
        st = _lib.Stats()
        _lib.check("sphfilt_plan_stats", self._lib.sphfilt_plan_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def set_schedule(self, theta_cols: int = 0, phi_lines: int = 0):
        _lib.check("sphfilt_plan_set_schedule",
                   self._lib.sphfilt_plan_set_schedule(self._h, int(theta_cols), int(phi_lines)))

    def get_schedule(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _lib.check("sphfilt_plan_get_schedule",
                   self._lib.sphfilt_plan_get_schedule(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


def lib():
    return _lib.load()
