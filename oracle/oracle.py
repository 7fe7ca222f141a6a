"""ctypes wrapper of the C oracle (sphfilt_oracle.c) -- TEST INFRASTRUCTURE ONLY.

Arrays are numpy float64, C order, shape (n_fields, n_r, n_theta, n_phi).
The per-field parameters follow the paper's filter (arXiv:2305.01537,
Sec. II.A): parity sign (-1)^a, rho = r/dr_min per shell, the cutoff scale
cal-L per field and the filter kind per field.
"""
import ctypes
import os

import numpy as np

EXP, GAUSS, SHARP, HYBRID = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libsphfilt_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            from .build import build
            build()
        lib = ctypes.CDLL(lib_path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        sig = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, dp, dp, ip,
               ctypes.c_double, dp]
        for name in ("orc_theta_pass", "orc_phi_pass", "orc_forward", "orc_adjoint"):
            fn = getattr(lib, name)
            fn.argtypes = sig
            fn.restype = ctypes.c_int
        lib.orc_mask.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_mask.restype = ctypes.c_double
        lib.orc_theta_cutoff.argtypes = [ctypes.c_double] * 3
        lib.orc_theta_cutoff.restype = ctypes.c_double
        lib.orc_phi_cutoff.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double]
        lib.orc_phi_cutoff.restype = ctypes.c_double
        lib.orc_sin_theta.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.orc_sin_theta.restype = ctypes.c_double
        lib.orc_set_detector.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_set_detector.restype = None
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_shock_detected.argtypes = [dp, ctypes.c_int]
        lib.orc_shock_detected.restype = ctypes.c_int
        ucp = ctypes.POINTER(ctypes.c_ubyte)
        lib.orc_theta_decisions.argtypes = [dp, ucp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ip, ip]
        lib.orc_theta_decisions.restype = ctypes.c_int
        lib.orc_phi_decisions.argtypes = [dp, ucp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ip]
        lib.orc_phi_decisions.restype = ctypes.c_int
        _lib = lib
    return _lib


def mask(kind: int, qhat: float, c: float) -> float:
    return _load().orc_mask(int(kind), float(qhat), float(c))


def theta_cutoff(rho: float, L: float, floor_modes: float = 2.0) -> float:
    return _load().orc_theta_cutoff(float(rho), float(L), float(floor_modes))


def phi_cutoff(rho: float, L: float, j: int, n_theta: int, floor_modes: float = 2.0) -> float:
    return _load().orc_phi_cutoff(float(rho), float(L), int(j), int(n_theta), float(floor_modes))


def sin_theta(j: int, n_theta: int) -> float:
    return _load().orc_sin_theta(int(j), int(n_theta))


def _params(x, parity, rho, L, kind):
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim != 4:
        raise ValueError("field array must have shape (n_fields, n_r, n_theta, n_phi)")
    F, R, T, P = x.shape
    parity = np.ascontiguousarray(np.broadcast_to(np.asarray(parity, dtype=np.int32), (F,)))
    if rho is None:
        rho = np.arange(R, dtype=np.float64) + 0.5
    rho = np.ascontiguousarray(np.broadcast_to(np.asarray(rho, dtype=np.float64), (R,)))
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (F,)))
    kind = np.ascontiguousarray(np.broadcast_to(np.asarray(kind, dtype=np.int32), (F,)))
    return x, parity, rho, L, kind


def _run(name, x, parity, rho, L, kind, floor_modes, return_imag):
    x, parity, rho, L, kind = _params(x, parity, rho, L, kind)
    out = np.empty_like(x)
    imag = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    rc = getattr(_load(), name)(
        x.ctypes.data_as(dp), out.ctypes.data_as(dp), *[ctypes.c_int(v) for v in x.shape],
        parity.ctypes.data_as(ip), rho.ctypes.data_as(dp), L.ctypes.data_as(dp),
        kind.ctypes.data_as(ip), ctypes.c_double(floor_modes), ctypes.byref(imag))
    if rc != 0:
        raise ValueError(f"{name} failed with status {rc}")
    return (out, imag.value) if return_imag else out


def theta_pass(x, parity=1, rho=None, L=3.0, kind=EXP, floor_modes=2.0, return_imag=False):
    """Theta filter alone (extension across the poles, FFT along vartheta, mask, iFFT)."""
    return _run("orc_theta_pass", x, parity, rho, L, kind, floor_modes, return_imag)


def phi_pass(x, parity=1, rho=None, L=3.0, kind=EXP, floor_modes=2.0, return_imag=False):
    """Phi filter alone (FFT along each ring, latitude-dependent mask, iFFT)."""
    return _run("orc_phi_pass", x, parity, rho, L, kind, floor_modes, return_imag)


def forward(x, parity=1, rho=None, L=3.0, kind=EXP, floor_modes=2.0, return_imag=False):
    """The double FFT filter: theta-pass, then phi-pass."""
    return _run("orc_forward", x, parity, rho, L, kind, floor_modes, return_imag)


def adjoint(x, parity=1, rho=None, L=3.0, kind=EXP, floor_modes=2.0, return_imag=False):
    """Transpose of the double FFT filter: phi-pass, then theta-pass."""
    return _run("orc_adjoint", x, parity, rho, L, kind, floor_modes, return_imag)


def set_detector(eps: float = 1e-12, threshold: float = 0.95) -> None:
    """Parameters of Jameson's detector used by the hybrid filter."""
    _load().orc_set_detector(float(eps), float(threshold))


def set_threads(n: int) -> int:
    """Threads of the oracle's loops over lines (0: all processors); returns the
    previous setting.  For timing only."""
    return int(_load().orc_set_threads(int(n)))


def shock_detected(line) -> bool:
    g = np.ascontiguousarray(line, dtype=np.float64)
    return bool(_load().orc_shock_detected(g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), g.size))


def decisions(x, parity=1, kind=HYBRID):
    """Hybrid choices (1 = Gaussian) of a theta-pass and of a phi-pass over x."""
    x, parity, _, _, kind = _params(x, parity, None, 1.0, kind)
    F, R, T, P = x.shape
    th = np.zeros((F, R, P // 2), dtype=np.uint8)
    ph = np.zeros((F, R, T), dtype=np.uint8)
    dp = ctypes.POINTER(ctypes.c_double)
    ucp = ctypes.POINTER(ctypes.c_ubyte)
    ip = ctypes.POINTER(ctypes.c_int)
    lib = _load()
    rc = lib.orc_theta_decisions(x.ctypes.data_as(dp), th.ctypes.data_as(ucp), F, R, T, P,
                                 parity.ctypes.data_as(ip), kind.ctypes.data_as(ip))
    rc |= lib.orc_phi_decisions(x.ctypes.data_as(dp), ph.ctypes.data_as(ucp), F, R, T, P,
                                kind.ctypes.data_as(ip))
    if rc:
        raise ValueError("decision export failed")
    return th, ph
