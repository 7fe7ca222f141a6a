"""The fused shell kernel on the GPU.

On grids with n_phi = 2 n_theta <= 128 a plan runs every shell whose theta
lines and rings are all filtered through one kernel that keeps the shell in
LDS between the two passes, in one launch with the ring pairs of the other
shells.  It runs the same line transforms as the two-pass path, packing other
meridian pairs into its complex theta lines (k and k + N/4, where the two-pass
kernel packs adjacent pairs), so the two agree to rounding, and both match the
oracle; in place and out of place run the same kernel and are bitwise equal.  The shapes
leave the number of fused shells ragged against the shells one workgroup takes
(8 at n_phi = 32, 2 at 64, 1 at 128) and mix fused shells with shells that
only the phi pass touches and shells that are left alone.
"""
import numpy as np
import pytest

import oracle
from paper_2305_01537_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12
EXP, GAUSS, SHARP, HYBRID = 0, 1, 2, 3

SHAPES = [(5, 13, 16, 32), (3, 9, 32, 64), (3, 13, 64, 128)]


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def fields(shape, seed):
    F, R, T, P = shape
    rng = np.random.default_rng(seed)
    theta, phi = synth.theta_grid(T), synth.phi_grid(P)
    x = np.empty(shape)
    for f in range(F):
        for i in range(R):
            x[f, i] = synth.angular_sum(rng, min(T // 2, 12), theta, phi, lambda l: 1.0 / (l + 1))
    x += 1e-3 * rng.standard_normal(shape)
    parity = np.where(rng.random(F) < 0.5, 1, -1).astype(np.int32)
    x[parity < 0] *= np.sin(theta)[None, :, None]
    return x, parity


def plan_for(shape, parity, L, kind=None):
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = shape
    return Plan(R, T, P, F, parity=parity, L=L, kind=kind)


def run(torch, plan, name, x, inplace):
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    fn = getattr(plan, name)
    y = fn(xd, out=xd) if inplace else fn(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("shape", SHAPES)
def test_fused_matches_the_two_pass_filter(torch_gpu, shape):
    torch = torch_gpu
    F, R, T, P = shape
    x, parity = fields(shape, 71 + T)
    kind = np.array([EXP, GAUSS, SHARP, EXP, EXP][:F], dtype=np.int32)
    # l_max = 2 rho cal-L < n_theta up to rho ~ T / (2 cal-L): with cal-L ~ T / R
    # the inner shells are fused, the outer ones only phi-filtered near the
    # poles (EXP/SHARP), and the Gaussian field is fused everywhere
    L = np.array([1.0, 0.9, 0.8, 1.3, 2.0][:F]) * (T / R)
    plan = plan_for(shape, parity, L, kind)
    st = plan.stats()
    enabled, n_fused = plan.get_fused()
    print(f"[gpu] fused {shape} shells fused {n_fused} of {F * R}", flush=True)
    assert enabled and n_fused == st["shells_fused"]
    assert 0 < n_fused < st["theta_shells_total"]
    assert st["theta_shells_active"] == n_fused
    for name in ("apply", "apply_adjoint"):
        plan.set_fused(True)
        a = run(torch, plan, name, x, False)
        assert np.array_equal(run(torch, plan, name, x, True), a), name
        plan.set_fused(False)
        b = run(torch, plan, name, x, False)
        assert rel(a, b) <= 1e-14, (name, rel(a, b))
    plan.set_fused(True)
    ref_f = oracle.forward(x, parity=parity, L=L, kind=kind)
    ref_a = oracle.adjoint(x, parity=parity, L=L, kind=kind)
    assert rel(run(torch, plan, "apply", x, False), ref_f) <= TOL
    assert rel(run(torch, plan, "apply_adjoint", x, True), ref_a) <= TOL
    plan.close()


@pytest.mark.parametrize("shape", [(2, 3, 16, 32), (1, 5, 32, 64), (2, 2, 64, 128)])
def test_every_shell_fused(torch_gpu, shape):
    # a small cutoff filters every line: all shells go through the fused kernel
    torch = torch_gpu
    F, R, T, P = shape
    x, parity = fields(shape, 81 + T)
    L = np.full(F, 0.2)
    plan = plan_for(shape, parity, L)
    assert plan.get_fused() == (True, F * R)
    for name, ref_fn in (("apply", oracle.forward), ("apply_adjoint", oracle.adjoint)):
        ref = ref_fn(x, parity=parity, L=L)
        out = run(torch, plan, name, x, False)
        assert rel(out, ref) <= TOL, name
        assert np.array_equal(run(torch, plan, name, x, True), out), name
    plan.close()


def test_fused_hybrid_decisions_and_replay(torch_gpu):
    torch = torch_gpu
    shape = (3, 4, 32, 64)
    x, _ = fields(shape, 91)
    x[:, :, :, :] += 3.0
    x[0, 1, :16, 0] = 0.0                                   # a theta jump
    x[0, 2, 3, :] = np.where(np.arange(64) < 21, 0.0, 2.0)  # a phi jump
    parity = np.array([1, 1, 1], dtype=np.int32)
    kind = np.array([HYBRID, HYBRID, EXP], dtype=np.int32)
    L = np.array([0.6, 0.9, 0.6])
    plan = plan_for(shape, parity, L, kind)
    assert plan.get_fused()[1] > 0
    res = {}
    for fused in (True, False):
        plan.set_fused(fused)
        th, ph = plan.decision_buffers()
        y = plan.apply_ex(torch.from_numpy(x).cuda(), theta_dec=th, phi_dec=ph)
        g = torch.from_numpy(np.random.default_rng(92).standard_normal(shape)).cuda()
        z = plan.apply_ex(g, adjoint=True, theta_dec=th, phi_dec=ph, replay=True)
        torch.cuda.synchronize()
        res[fused] = (y.cpu().numpy(), th.cpu().numpy(), ph.cpu().numpy(), z.cpu().numpy())
    # the same decisions (nothing here sits within rounding of the threshold)
    assert np.array_equal(res[True][1], res[False][1])
    assert np.array_equal(res[True][2], res[False][2])
    assert rel(res[True][0], res[False][0]) <= 1e-14
    assert rel(res[True][3], res[False][3]) <= 1e-14
    y, th, ph, _ = res[True]
    assert th.any() and ph.any()
    ref = oracle.forward(x, parity=parity, L=L, kind=kind)
    assert rel(y, ref) <= TOL
    th_o, _ = oracle.decisions(x, parity=parity, kind=kind)
    assert np.array_equal(th, th_o)
    plan.close()


def test_set_fused_rejects_bad_values(torch_gpu):
    from paper_2305_01537_amd import _lib
    x, parity = fields((1, 2, 16, 32), 5)
    plan = plan_for(x.shape, parity, np.array([0.2]))
    lib = _lib.load()
    assert lib.sphfilt_plan_set_fused(plan._h, 2) == _lib.EINVAL
    assert lib.sphfilt_plan_set_fused(None, 1) == _lib.EINVAL
    plan.set_fused(False)
    assert plan.get_fused() == (False, 0)
    plan.close()
