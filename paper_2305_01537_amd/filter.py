"""Python binding of the double FFT filter (argument marshalling only).

Every step of the filter runs in libsphfilt.so's HIP kernels; this module
checks tensor shapes and dtypes, passes raw device pointers and the current
HIP stream through the C-ABI, and raises on a non-zero status.  PyTorch
provides device memory and streams.

The operator (arXiv:2305.01537, Sec. II.A): theta-filter on lines extended
across the poles, then phi-filter on rings, with cutoffs l_max = max(2, 2 rho L)
and m_max = max(2, 2 rho sin(theta) L).  Its transpose is the phi-pass
followed by the theta-pass; SphFilter uses it as the backward.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (EXP, GAUSS, HYBRID, SHARP, THETA_FFT, THETA_MFMA, SphfiltError,  # noqa: F401
                   status_string)


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

    def __init__(self, n_r, n_fields, parity, L, rho, kind, floor_modes, detector_eps=0.0,
                 detector_threshold=0.0):
        self.parity = _as_int_array(parity, n_fields, "parity")
        self.L = _as_double_array(L, n_fields, "L")
        self.rho = None if rho is None else _as_double_array(rho, n_r, "rho")
        self.kind = None if kind is None else _as_int_array(kind, n_fields, "kind")
        self.cut = _lib.Cutoff(
            None if self.rho is None else self.rho.ctypes.data_as(_lib.c_double_p),
            self.L.ctypes.data_as(_lib.c_double_p),
            None if self.kind is None else self.kind.ctypes.data_as(_lib.c_int_p),
            float(floor_modes), float(detector_eps), float(detector_threshold))
        self.has_hybrid = self.kind is not None and bool((self.kind == HYBRID).any())

    @property
    def parity_p(self):
        return self.parity.ctypes.data_as(_lib.c_int_p)


def workload_stats(n_r, n_theta, n_phi, n_fields, parity=1, L=3.0, rho=None, kind=None,
                   floor_modes=2.0, detector_eps=0.0, detector_threshold=0.0) -> dict:
    """Active lines and algorithmic HBM bytes of a filter call (host only)."""
    prm = _Params(n_r, n_fields, parity, L, rho, kind, floor_modes, detector_eps,
                  detector_threshold)
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
    rho: r/dr_min per shell (None: i + 1/2); kind: EXP/GAUSS/SHARP/HYBRID per
    field (None: EXP); floor_modes: the cutoff floor (2 in the paper);
    detector_eps / detector_threshold: Jameson's detector of the HYBRID kind
    (0: the defaults 1e-12 and 0.95).
    The plan's tables live on the current HIP device.
    """

    def __init__(self, n_r: int, n_theta: int, n_phi: int, n_fields: int, parity=1, L=3.0,
                 rho=None, kind=None, floor_modes: float = 2.0, detector_eps: float = 0.0,
                 detector_threshold: float = 0.0):
        self.shape = (int(n_fields), int(n_r), int(n_theta), int(n_phi))
        self._prm = _Params(n_r, n_fields, parity, L, rho, kind, floor_modes, detector_eps,
                            detector_threshold)
        self.has_hybrid = self._prm.has_hybrid
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

    def decision_buffers(self, device="cuda"):
        """Zeroed byte buffers for the hybrid kind's decisions: one per extended
        theta line [F][n_r][n_phi/2] and one per ring [F][n_r][n_theta]."""
        import torch
        F, R, T, P = self.shape
        return (torch.zeros((F, R, P // 2), dtype=torch.uint8, device=device),
                torch.zeros((F, R, T), dtype=torch.uint8, device=device))

    def apply_ex(self, x, out=None, adjoint=False, theta_dec=None, phi_dec=None, replay=False,
                 stream=None):
        """The filter (adjoint=True: its transpose) with the hybrid decisions
        recorded into (replay=False) or taken from (replay=True) the buffers."""
        import torch
        self._check_tensor(x, "x")
        if out is None:
            out = torch.empty_like(x)
        else:
            self._check_tensor(out, "out")
        F, R, T, P = self.shape
        for buf, shp, name in ((theta_dec, (F, R, P // 2), "theta_dec"), (phi_dec, (F, R, T), "phi_dec")):
            if buf is not None and (buf.dtype != torch.uint8 or tuple(buf.shape) != shp or
                                    buf.device.type != "cuda" or not buf.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous uint8 HIP tensor of shape {shp}")
        ptr = lambda b: ctypes.c_void_p(b.data_ptr()) if b is not None else None
        rc = self._lib.sphfilt_apply_ex(self._h, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), 1 if adjoint else 0,
                                        ptr(theta_dec), ptr(phi_dec), 1 if replay else 0,
                                        _stream_handle(x, stream))
        _lib.check("sphfilt_apply_ex", rc)
        return out

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

    def set_fused(self, enable: bool):
        """Fuse the shells the grid allows (n_phi = 2 n_theta in {32, 64, 128}) or always
        run two passes; see sphfilt_plan_set_fused."""
        _lib.check("sphfilt_plan_set_fused", self._lib.sphfilt_plan_set_fused(self._h, int(bool(enable))))

    def tune(self, cache_path: Optional[str] = None):
        """Autotune the plan's launch settings (see sphfilt_plan_tune);
        returns {"tuned_us", "default_us"}."""
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check("sphfilt_plan_tune", self._lib.sphfilt_plan_tune(self._h, path))
        a, b = ctypes.c_double(), ctypes.c_double()
        _lib.check("sphfilt_plan_tuned_times",
                   self._lib.sphfilt_plan_tuned_times(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"tuned_us": a.value, "default_us": b.value}

    def set_theta_variant(self, variant: int):
        """THETA_FFT (default) or THETA_MFMA: the theta pass as the circulant
        product on the matrix cores (grids with n_phi = 2 n_theta in {32, 64});
        see sphfilt_plan_set_theta_variant."""
        _lib.check("sphfilt_plan_set_theta_variant",
                   self._lib.sphfilt_plan_set_theta_variant(self._h, int(variant)))

    def get_theta_variant(self) -> int:
        a = ctypes.c_int()
        _lib.check("sphfilt_plan_get_theta_variant",
                   self._lib.sphfilt_plan_get_theta_variant(self._h, ctypes.byref(a)))
        return a.value

    def set_overlap(self, mode: int):
        """In place, run the rings that do not depend on the theta pass on a
        second stream of the plan: 0 never (the default), 1 when they move
        >= 128 MiB, 2 always; see sphfilt_plan_set_overlap."""
        _lib.check("sphfilt_plan_set_overlap", self._lib.sphfilt_plan_set_overlap(self._h, int(mode)))

    def get_overlap(self) -> int:
        a = ctypes.c_int()
        _lib.check("sphfilt_plan_get_overlap", self._lib.sphfilt_plan_get_overlap(self._h, ctypes.byref(a)))
        return a.value

    def get_fused(self):
        """(enabled, number of shells fused)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _lib.check("sphfilt_plan_get_fused",
                   self._lib.sphfilt_plan_get_fused(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), b.value


class Batch:
    """Many uneven spherical patches filtered by one graph-replayed launch.

    patches: a sequence of objects or dicts with n_r, n_theta, n_phi, n_fields,
    parity, L and optionally rho, kind, floor_modes (as for Plan).
    tune_cache: path of a JSON schedule cache; None = default schedule.  A
    patch set not yet in the cache is autotuned (on scratch fields) at
    creation and recorded.
    Each patch is filtered exactly as by its own Plan (bit-identical results).
    """

    def __init__(self, patches, tune_cache: Optional[str] = None):
        def get(p, k, d=None):
            return p.get(k, d) if isinstance(p, dict) else getattr(p, k, d)
        self.shapes = []
        self._prms = []
        n = len(patches)
        if n == 0:
            raise ValueError("a batch needs at least one patch")
        descs = (_lib.PatchDesc * n)()
        for i, p in enumerate(patches):
            F, R, T, P = (int(get(p, "n_fields")), int(get(p, "n_r")), int(get(p, "n_theta")),
                          int(get(p, "n_phi")))
            prm = _Params(R, F, get(p, "parity", 1), get(p, "L", 3.0), get(p, "rho"),
                          get(p, "kind"), get(p, "floor_modes", 2.0), get(p, "detector_eps", 0.0),
                          get(p, "detector_threshold", 0.0))
            self._prms.append(prm)
            self.shapes.append((F, R, T, P))
            descs[i].n_r, descs[i].n_theta, descs[i].n_phi, descs[i].n_fields = R, T, P, F
            descs[i].parity = prm.parity_p
            descs[i].cut = prm.cut
        self._descs = descs
        lib = _lib.load()
        h = ctypes.c_void_p()
        path = None if tune_cache is None else str(tune_cache).encode()
        _lib.check("sphfilt_batch_create", lib.sphfilt_batch_create(ctypes.byref(h), n, descs, path))
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.sphfilt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.shapes)

    @property
    def handle(self):
        return self._h

    def _pointers(self, xs, outs):
        import torch
        if len(xs) != len(self.shapes):
            raise ValueError(f"expected {len(self.shapes)} tensors")
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for x, o, shp in zip(xs, outs, self.shapes):
            for t, name in ((x, "input"), (o, "output")):
                if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or \
                        t.device.type != "cuda" or tuple(t.shape) != shp or not t.is_contiguous():
                    raise ValueError(f"{name} must be a contiguous float64 HIP tensor of shape {shp}")
        n = len(xs)
        ins_p = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        outs_p = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        return outs, ins_p, outs_p

    def apply(self, xs, outs=None, adjoint: bool = False, stream=None, check: bool = False):
        """outs[p] = F xs[p] (or F^T with adjoint=True); outs=xs filters in place.

        check=True synchronises the device after the call and raises if the
        batch kernel flagged an error (a second-pass item that gave up waiting
        for its shells; see status())."""
        outs, ins_p, outs_p = self._pointers(xs, outs)
        rc = self._lib.sphfilt_batch_apply(self._h, ins_p, outs_p, 1 if adjoint else 0,
                                           _stream_handle(xs[0], stream))
        _lib.check("sphfilt_batch_apply", rc)
        if check:
            err = self.status()
            if err:
                raise SphfiltError("sphfilt_batch_apply (device error word)", _lib.EDEVICE)
        return outs

    def apply_noalloc(self, xs, outs=None, adjoint: bool = False, stream=None):
        """The same filter through sphfilt_batch_apply_noalloc: no device
        allocation during the call (the per-call state lives in the library's
        static device array; calls on one device must not overlap)."""
        outs, ins_p, outs_p = self._pointers(xs, outs)
        rc = self._lib.sphfilt_batch_apply_noalloc(self._h, ins_p, outs_p, 1 if adjoint else 0,
                                                   _stream_handle(xs[0], stream))
        _lib.check("sphfilt_batch_apply_noalloc", rc)
        return outs

    def tune(self, cache_path: Optional[str] = None):
        path = None if cache_path is None else str(cache_path).encode()
        _lib.check("sphfilt_batch_tune", self._lib.sphfilt_batch_tune(self._h, path))

    def set_schedule(self, split: int, workgroups_per_cu: int):
        _lib.check("sphfilt_batch_set_schedule",
                   self._lib.sphfilt_batch_set_schedule(self._h, int(split), int(workgroups_per_cu)))

    def get_schedule(self):
        """The whole schedule (see sphfilt_batch_schedule): split,
        workgroups_per_cu, fused, theta_tiles, phi_groups, theta_cols
        ({line length: width} for the tuned widths), tuned_us, default_us."""
        q = _lib.BatchSchedule()
        _lib.check("sphfilt_batch_get_schedule_ex",
                   self._lib.sphfilt_batch_get_schedule_ex(self._h, ctypes.byref(q)))
        return {"split": q.split, "workgroups_per_cu": q.workgroups_per_cu, "fused": q.fused,
                "theta_tiles": q.theta_tiles, "phi_groups": q.phi_groups,
                "theta_cols": {n: q.theta_cols[i] for i, n in enumerate(_lib.THETA_LINES)
                               if q.theta_cols[i]},
                "tuned_us": q.tuned_us, "default_us": q.default_us}

    def set_schedule_ex(self, split: int = 0, workgroups_per_cu: int = -1, fused: bool = True,
                        theta_tiles: int = 1, phi_groups: int = 1, theta_cols=None):
        """Set every schedule knob at once; theta_cols: {theta line length:
        sub-tile width} (others keep their default width)."""
        q = _lib.BatchSchedule()
        q.split, q.workgroups_per_cu, q.fused = int(split), int(workgroups_per_cu), int(bool(fused))
        q.theta_tiles, q.phi_groups = int(theta_tiles), int(phi_groups)
        for n, w in (theta_cols or {}).items():
            q.theta_cols[_lib.THETA_LINES.index(int(n))] = int(w)
        _lib.check("sphfilt_batch_set_schedule_ex",
                   self._lib.sphfilt_batch_set_schedule_ex(self._h, ctypes.byref(q)))

    def status(self) -> int:
        e = ctypes.c_int()
        _lib.check("sphfilt_batch_status", self._lib.sphfilt_batch_status(self._h, ctypes.byref(e)))
        return e.value

    def stats(self) -> dict:
        st = _lib.Stats()
        _lib.check("sphfilt_batch_stats", self._lib.sphfilt_batch_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def set_fused(self, enable: bool):
        """Fused items for patches whose shells fit in LDS (the default), or
        every patch in two passes; see sphfilt_batch_set_fused."""
        _lib.check("sphfilt_batch_set_fused", self._lib.sphfilt_batch_set_fused(self._h, int(bool(enable))))

    def get_fused(self):
        """(enabled, number of shells fused)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _lib.check("sphfilt_batch_get_fused",
                   self._lib.sphfilt_batch_get_fused(self._h, ctypes.byref(a), ctypes.byref(b)))
        return bool(a.value), b.value


def lib():
    return _lib.load()
