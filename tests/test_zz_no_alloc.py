"""The allocation-free batch entry point, sphfilt_batch_apply_noalloc.

It runs the same kernels on the same work lists as sphfilt_batch_apply, with
the per-call counters, tickets, error word and pointer tables in the
library's static device array instead of the batch's own memory, so its
output must equal sphfilt_batch_apply's bit for bit, and both must match the
oracle.  Two calls in a row, the second on a smaller batch, check that each
call clears the array's state left by the previous one.  The size limits are
rejected on the host, before any device call.
"""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2305_01537_amd import _lib

pytestmark = pytest.mark.gpu


def make_patches(shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for F, R, T, P in shapes:
        out.append(dict(n_fields=F, n_r=R, n_theta=T, n_phi=P,
                        parity=rng.choice([1, -1], F).astype(np.int32),
                        L=rng.choice([0.3, 0.8, 3.0], F),
                        kind=rng.choice([0, 1, 2], F).astype(np.int32),
                        rho=0.5 + np.arange(R) * rng.uniform(0.5, 2.0),
                        x=rng.standard_normal((F, R, T, P))))
    return out


def c_call(fname, batch, xs, outs, adjoint):
    """One call through the C-ABI (ctypes), on torch's current stream."""
    import torch
    n = len(xs)
    ins_p = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
    outs_p = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(_lib.load(), fname)(batch.handle, ins_p, outs_p, 1 if adjoint else 0, stream)


def oracle_out(p, adjoint):
    fn = oracle.adjoint if adjoint else oracle.forward
    return fn(p["x"], parity=p["parity"], rho=p["rho"], L=p["L"], kind=p["kind"])


def run_pair(torch, patches, schedule, adjoint, inplace):
    """(noalloc outputs, graph-path outputs) on the same inputs."""
    from paper_2305_01537_amd.filter import Batch
    batch = Batch(patches)
    batch.set_schedule(*schedule)
    res = []
    for fname in ("sphfilt_batch_apply_noalloc", "sphfilt_batch_apply"):
        xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
        outs = xs if inplace else [torch.full_like(x, np.nan) for x in xs]
        rc = c_call(fname, batch, xs, outs, adjoint)
        assert rc == _lib.OK, (fname, rc)
        torch.cuda.synchronize()
        res.append([o.cpu().numpy() for o in outs])
    batch.close()
    return res


@pytest.mark.parametrize("schedule", [(0, -1), (1, 0), (2, -1)],
                         ids=["one-kernel-deps", "two-kernels-persistent", "side-branch"])
def test_noalloc_equals_batch_apply_two_calls(schedule):
    import torch
    big = make_patches([(3, 9, 16, 32), (2, 6, 32, 64), (4, 5, 64, 128), (2, 4, 128, 256),
                        (1, 3, 64, 32), (3, 7, 32, 128)], seed=71)
    small = make_patches([(2, 3, 32, 64), (1, 2, 16, 32)], seed=72)
    for patches, adjoint, inplace in ((big, False, False), (small, True, True)):
        got, ref = run_pair(torch, patches, schedule, adjoint, inplace)
        for p, g, r in zip(patches, got, ref):
            assert np.array_equal(g, r), "noalloc differs from sphfilt_batch_apply"
            want = oracle_out(p, adjoint)
            err = np.abs(g - want).max() / np.abs(want).max()
            assert err <= 1e-12, err


def test_noalloc_hybrid_and_mixed_radix_patches():
    """The other kernel instances through the allocation-free call: hybrid fields
    (the detector decides from the data) and lines of 48, 96 and 160 points,
    two calls in a row, the second on a smaller batch."""
    import torch
    big = make_patches([(3, 5, 24, 48), (2, 4, 48, 96), (2, 3, 80, 160), (3, 4, 64, 128)], seed=73)
    small = make_patches([(2, 3, 24, 48)], seed=74)
    for patches in (big, small):
        for p in patches:
            p["kind"][0] = 3
            p["x"][0] += 2.0
            p["x"][0, 0, :, : p["n_phi"] // 3] = 0.0          # a jump for the detector
    for patches, adjoint, inplace in ((big, False, True), (small, True, False)):
        got, ref = run_pair(torch, patches, (1, -1), adjoint, inplace)
        for p, g, r in zip(patches, got, ref):
            assert np.array_equal(g, r), "noalloc differs from sphfilt_batch_apply"
            want = oracle_out(p, adjoint)
            err = np.abs(g - want).max() / np.abs(want).max()
            assert err <= 1e-12, err


def test_noalloc_rejects_sizes_beyond_the_array():
    """More patches or shells than the static array holds: SPHFILT_EUNSUPPORTED,
    decided on the host before any device call (the pointers passed are
    aligned, non-overlapping addresses that are never dereferenced)."""
    import torch  # noqa: F401  (initialises the device the batch is made on)
    from paper_2305_01537_amd.filter import Batch
    cases = [[dict(n_fields=1, n_r=1, n_theta=16, n_phi=32, parity=1, L=3.0)] * 1025,
             [dict(n_fields=1, n_r=262145, n_theta=16, n_phi=32, parity=1, L=3.0)]]
    for patches in cases:
        batch = Batch(patches)
        n = len(patches)
        size = 8 * patches[0]["n_r"] * 16 * 32
        base = 1 << 40
        ins_p = (ctypes.c_void_p * n)(*[base + i * size for i in range(n)])
        outs_p = (ctypes.c_void_p * n)(*[base + i * size for i in range(n)])
        rc = _lib.load().sphfilt_batch_apply_noalloc(batch.handle, ins_p, outs_p, 0, None)
        assert rc == _lib.EUNSUPPORTED
        batch.close()
