"""sphfilt: the double FFT filter of arXiv:2305.01537 on MI355X (gfx950).

The filter runs in hand-written HIP kernels behind a C-ABI library
(`libsphfilt.so`, declared in include/sphfilt.h).  This package is the thin
Python binding over it; PyTorch supplies device memory and streams only.
The binding is imported lazily so that `synth` can be used without a GPU.
"""
__all__ = ["synth"]


def __getattr__(name):
    if name in ("Plan", "Batch", "lib", "workload_stats", "SphfiltError", "status_string"):
        from . import filter as _f
        return getattr(_f, name)
    if name in ("SphFilter", "sph_filter", "filter_chain"):
        from . import autograd as _a
        return getattr(_a, name)
    raise AttributeError(name)
