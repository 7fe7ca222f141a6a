"""ctypes declarations of libsphfilt.so (include/sphfilt.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphfilt.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4
EXP, GAUSS, SHARP, HYBRID = 0, 1, 2, 3
THETA_FFT, THETA_MFMA = 0, 1

c_int_p = ctypes.POINTER(ctypes.c_int)
c_double_p = ctypes.POINTER(ctypes.c_double)


class Cutoff(ctypes.Structure):
    _fields_ = [("rho", c_double_p), ("L", c_double_p), ("kind", c_int_p),
                ("floor_modes", ctypes.c_double), ("detector_eps", ctypes.c_double),
                ("detector_threshold", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in (
        "n_points", "theta_shells_total", "theta_shells_active", "theta_lines_total",
        "theta_lines_active", "phi_rings_total", "phi_rings_active", "bytes_forward_inplace",
        "bytes_forward_outofplace", "bytes_adjoint_inplace", "bytes_adjoint_outofplace",
        "shells_fused", "bytes_fused_inplace")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class BatchSchedule(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int), ("workgroups_per_cu", ctypes.c_int), ("fused", ctypes.c_int),
                ("theta_tiles", ctypes.c_int), ("phi_groups", ctypes.c_int),
                ("theta_cols", ctypes.c_int * 9), ("tuned_us", ctypes.c_double),
                ("default_us", ctypes.c_double)]


THETA_LINES = (32, 48, 64, 80, 96, 128, 160, 192, 256)


class PatchDesc(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int), ("n_theta", ctypes.c_int), ("n_phi", ctypes.c_int),
                ("n_fields", ctypes.c_int), ("parity", c_int_p), ("cut", Cutoff)]


# name -> (restype, argtypes)
SIGNATURES = {
    "sphfilt_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int, c_int_p, ctypes.POINTER(Cutoff)]),
    "sphfilt_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sphfilt_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sphfilt_apply_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sphfilt_apply_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "sphfilt_apply_theta": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sphfilt_apply_phi": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sphfilt_plan_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "sphfilt_workload_stats": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              c_int_p, ctypes.POINTER(Cutoff), ctypes.POINTER(Stats)]),
    "sphfilt_plan_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "sphfilt_plan_get_schedule": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p]),
    "sphfilt_plan_set_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sphfilt_plan_get_fused": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p]),
    "sphfilt_plan_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "sphfilt_plan_tuned_times": (ctypes.c_int, [ctypes.c_void_p, c_double_p, c_double_p]),
    "sphfilt_plan_set_theta_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sphfilt_plan_get_theta_variant": (ctypes.c_int, [ctypes.c_void_p, c_int_p]),
    "sphfilt_plan_set_overlap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sphfilt_plan_get_overlap": (ctypes.c_int, [ctypes.c_void_p, c_int_p]),
    "sphfilt_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                            ctypes.POINTER(PatchDesc), ctypes.c_char_p]),
    "sphfilt_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sphfilt_batch_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "sphfilt_batch_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                                   ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                                   ctypes.c_void_p]),
    "sphfilt_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "sphfilt_batch_set_schedule": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "sphfilt_batch_get_schedule": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p, c_double_p]),
    "sphfilt_batch_set_schedule_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchSchedule)]),
    "sphfilt_batch_get_schedule_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchSchedule)]),
    "sphfilt_batch_status": (ctypes.c_int, [ctypes.c_void_p, c_int_p]),
    "sphfilt_batch_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "sphfilt_batch_set_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "sphfilt_batch_get_fused": (ctypes.c_int, [ctypes.c_void_p, c_int_p, c_int_p]),
    "sphfilt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sphfilt_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libsphfilt.so once; raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2305_01537_amd.build` "
                              "(the filter has no non-HIP implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def status_string(code: int) -> str:
    return load().sphfilt_status_string(int(code)).decode()


class SphfiltError(RuntimeError):
    def __init__(self, where: str, code: int):
        self.code = int(code)
        super().__init__(f"{where}: {status_string(code)} (status {code})")


def check(where: str, code: int) -> None:
    if code != OK:
        raise SphfiltError(where, code)
