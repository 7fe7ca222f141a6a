"""Error paths that need a device: injected launch failures and the batch
kernel's bounded wait giving up.

Both are forced from the host (the SPHFILT_FAULT environment variable, read on
every call): a launch failure makes the entry points return SPHFILT_EDEVICE
before they enqueue anything; the wait fault raises every wait target of the
one-kernel batch schedule by one and cuts the spin short, so every
second-pass item gives up after a few polls, flags the device error word and
leaves its output as the first pass wrote it -- every kernel still runs to
its end.
"""
import ctypes

import numpy as np
import pytest

from paper_2305_01537_amd import _lib

pytestmark = pytest.mark.gpu


def small_patches(seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for F, R, T, P in ((2, 5, 32, 128), (3, 4, 64, 64), (1, 6, 16, 64)):
        out.append(dict(n_fields=F, n_r=R, n_theta=T, n_phi=P,
                        parity=rng.choice([1, -1], F).astype(np.int32), L=np.full(F, 0.4),
                        x=rng.standard_normal((F, R, T, P))))
    return out


def test_launch_fault_gives_edevice(monkeypatch):
    import torch
    from paper_2305_01537_amd.filter import Batch, Plan
    lib = _lib.load()
    p = small_patches()[0]
    plan = Plan(p["n_r"], p["n_theta"], p["n_phi"], p["n_fields"], parity=p["parity"], L=p["L"])
    batch = Batch(small_patches())
    x = torch.from_numpy(p["x"]).cuda()
    xs = [torch.from_numpy(q["x"]).cuda() for q in small_patches()]
    before = [t.clone() for t in xs]
    n = len(xs)
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    monkeypatch.setenv("SPHFILT_FAULT", "launch")
    xp = ctypes.c_void_p(x.data_ptr())
    assert lib.sphfilt_apply(plan.handle, xp, xp, stream) == _lib.EDEVICE
    assert lib.sphfilt_apply_adjoint(plan.handle, xp, xp, stream) == _lib.EDEVICE
    assert lib.sphfilt_batch_apply(batch.handle, ptrs, ptrs, 0, stream) == _lib.EDEVICE
    assert lib.sphfilt_batch_apply_noalloc(batch.handle, ptrs, ptrs, 0, stream) == _lib.EDEVICE
    monkeypatch.delenv("SPHFILT_FAULT")
    torch.cuda.synchronize()
    # nothing was enqueued: the fields are untouched, and calls work again
    assert torch.equal(x.cpu(), torch.from_numpy(p["x"]))
    for a, b in zip(xs, before):
        assert torch.equal(a, b)
    assert lib.sphfilt_batch_apply(batch.handle, ptrs, ptrs, 0, stream) == _lib.OK
    torch.cuda.synchronize()
    assert batch.status() == 0
    plan.close()
    batch.close()


@pytest.mark.parametrize("noalloc", [False, True])
def test_batch_wait_gives_up_and_skips_the_item(monkeypatch, noalloc):
    """One kernel with per-shell dependencies (split 0), forward, out of place:
    with every wait made unreachable, every phi item gives up, so each output
    is the theta pass alone (bitwise what a plan's theta pass gives) and the
    error word is set; apply(check=True) raises.  Without the fault the same
    batch gives the full filter and a clean status."""
    import torch
    from paper_2305_01537_amd.filter import Batch, Plan
    patches = small_patches()
    batch = Batch(patches)
    batch.set_fused(False)
    batch.set_schedule(0, -1)
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    theta_only, full = [], []
    for p, x in zip(patches, xs):
        plan = Plan(p["n_r"], p["n_theta"], p["n_phi"], p["n_fields"], parity=p["parity"], L=p["L"])
        plan.set_fused(False)
        theta_only.append(plan.apply_theta(x).cpu())
        full.append(plan.apply(x).cpu())
        plan.close()
    monkeypatch.setenv("SPHFILT_FAULT", "wait")
    outs = [torch.full_like(x, np.nan) for x in xs]
    if noalloc:
        batch.apply_noalloc(xs, outs)
    else:
        with pytest.raises(_lib.SphfiltError):
            batch.apply(xs, outs, check=True)
    torch.cuda.synchronize()
    assert batch.status() == 1
    for o, t in zip(outs, theta_only):
        assert torch.equal(o.cpu(), t)
    monkeypatch.delenv("SPHFILT_FAULT")
    outs = [torch.full_like(x, np.nan) for x in xs]
    (batch.apply_noalloc if noalloc else batch.apply)(xs, outs)
    torch.cuda.synchronize()
    assert batch.status() == 0
    for o, f in zip(outs, full):
        assert torch.equal(o.cpu(), f)
    batch.close()
