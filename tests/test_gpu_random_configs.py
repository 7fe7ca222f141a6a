"""Seeded sweep over plan configurations, against the oracle.

Each case draws a grid (2 n_theta and n_phi among the supported line lengths,
radix-3 and radix-5 ones included, so grids with fused shells, with overlapped passes and
plain ones all occur),
per-field kinds (exponential, Gaussian, sharp, hybrid) and parities, cut-off
scales over two decades, a radius table (uniform, stretched or None), a floor,
the call (forward or adjoint, in place or out of place) and the schedule
(fused shells and overlap on or off, theta tile and ring pairs per
workgroup).  The result must match the oracle to 1e-12 relative max-norm, and
the same call with the plain two-pass schedule to 1e-14.  With field 0 made
hybrid, recorded and replayed decisions give bitwise the same field and equal
the oracle's decisions.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12
LINES = (32, 48, 64, 80, 96, 128, 160, 192, 256)


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def draw(seed):
    rng = np.random.default_rng(1000 + seed)
    n_phi = int(rng.choice(LINES))
    # half the cases with n_phi = 2 n_theta (fused shells / overlap), the rest mixed
    n_theta = n_phi // 2 if rng.random() < 0.5 else int(rng.choice(LINES)) // 2
    F = int(rng.integers(1, 5))
    R = int(rng.integers(1, 9))
    while F * R * n_theta * n_phi > 300_000:
        R = max(1, R // 2)
        F = max(1, F - 1) if R == 1 else F
    kind = rng.choice([0, 0, 1, 2, 3], F).astype(np.int32)
    parity = rng.choice([1, -1], F).astype(np.int32)
    L = np.exp(rng.uniform(np.log(0.1), np.log(20.0), F))
    rho_kind = rng.integers(0, 3)
    rho = None if rho_kind == 0 else (0.5 + np.arange(R) * rng.uniform(0.3, 3.0) if rho_kind == 1
                                      else np.cumsum(rng.uniform(0.2, 5.0, R)))
    floor = float(rng.choice([2.0, 0.5, 3.5]))
    x = rng.standard_normal((F, R, n_theta, n_phi))
    x += 2.0 * (kind == 3)[:, None, None, None]                    # hybrid fields: level 2 ...
    hyb = np.flatnonzero(kind == 3)
    if hyb.size:                                                     # ... with a jump somewhere
        f = int(hyb[0])
        x[f, int(rng.integers(R)), int(rng.integers(n_theta)), : n_phi // 3] = 0.0
    call = dict(adjoint=bool(rng.random() < 0.5), inplace=bool(rng.random() < 0.5),
                fused=bool(rng.random() < 0.7), overlap=int(rng.choice([0, 1, 2])))
    return x, parity, kind, L, rho, floor, call


# lanes per line in the kernels (the second factor of the line's split)
LANES = {32: 4, 48: 4, 64: 8, 80: 8, 96: 8, 128: 8, 160: 16, 192: 16, 256: 16}


def draw_shape(seed, n_theta, n_phi):
    """A launch shape the plan accepts: theta_cols in {4..64}, at most n_phi/4
    and one theta workgroup's lines, with 2 theta_cols dividing n_phi/2;
    phi_lines in {4..64} with at most 256 lanes per workgroup.  Drawn from a
    generator of its own, so the rest of the case does not depend on it."""
    rng = np.random.default_rng(5000 + seed)
    n = 2 * n_theta
    cap = 256 // LANES[n]
    cols = [c for c in (4, 8, 16, 32, 64) if c <= n_phi // 4 and c <= cap and (n_phi // 2) % (2 * c) == 0]
    lines = [q for q in (4, 8, 16, 32, 64) if q * LANES[n_phi] <= 256]
    return int(rng.choice(cols)), int(rng.choice(lines))


def run(torch, plan, x, call):
    xd = torch.from_numpy(x).cuda()
    fn = plan.apply_adjoint if call["adjoint"] else plan.apply
    y = fn(xd, out=xd) if call["inplace"] else fn(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def rel(a, b, x):
    """Max-norm of a - b relative to the larger of b's max-norm and 1 % of the
    input x's.  A filtered field can vanish exactly (an odd-parity field whose
    kept modes are theta mode 0 and ring mode 0 only: the two halves of each
    extended line cancel), and then only the round-off of either side is left
    to compare; results that do not vanish stay above 0.4 % of the input's
    max-norm over these draws, so for them the bar is the plain relative one."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-2 * np.abs(x).max(), 1e-300))


@pytest.mark.parametrize("seed", range(240))
def test_random_configuration(torch_gpu, seed):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    x, parity, kind, L, rho, floor, call = draw(seed)
    F, R, T, P = x.shape
    print(f"[gpu] case {seed}: {x.shape} kind {kind.tolist()} {call}", flush=True)
    plan = Plan(R, T, P, F, parity=parity, L=L, rho=rho, kind=kind, floor_modes=floor)
    default_shape = plan.get_schedule()
    shape = draw_shape(seed, T, P)
    print(f"[gpu] case {seed}: launch shape {shape}", flush=True)
    plan.set_schedule(*shape)
    plan.set_fused(call["fused"])
    plan.set_overlap(call["overlap"])
    got = run(torch, plan, x, call)
    ref_fn = oracle.adjoint if call["adjoint"] else oracle.forward
    ref = ref_fn(x, parity=parity, rho=rho, L=L, kind=kind, floor_modes=floor)
    assert rel(got, ref, x) <= TOL, (seed, rel(got, ref, x))
    # the plain schedule: both passes on the caller's stream, no fused shells,
    # the default launch shape
    plan.set_schedule(*default_shape)
    plan.set_fused(False)
    plan.set_overlap(0)
    plain = run(torch, plan, x, call)
    assert rel(got, plain, x) <= 1e-14, (seed, rel(got, plain, x))
    plan.close()


@pytest.mark.parametrize("seed", range(64))
def test_random_hybrid_record_and_replay(torch_gpu, seed):
    """The same draws with field 0 made hybrid (level 2 added, so its lines mix
    smooth stretches and the jumps of the noise): recording the detector's
    decisions and replaying them gives bitwise the same field, the field
    matches the oracle, and every recorded decision of a hybrid field equals
    the oracle's (theta decisions on the first pass's input, phi decisions on
    the theta-filtered field, or the reverse for the adjoint)."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    x, parity, kind, L, rho, floor, call = draw(seed)
    kind = kind.copy()
    kind[0] = 3
    x = x.copy()
    x[0] += 2.0
    F, R, T, P = x.shape
    print(f"[gpu] hybrid record/replay case {seed}: {x.shape} kind {kind.tolist()} {call}", flush=True)
    plan = Plan(R, T, P, F, parity=parity, L=L, rho=rho, kind=kind, floor_modes=floor)
    plan.set_fused(call["fused"])
    plan.set_overlap(call["overlap"])
    adj = call["adjoint"]
    th, ph = plan.decision_buffers()
    xd = torch.from_numpy(x).cuda()
    rec = plan.apply_ex(xd, adjoint=adj, theta_dec=th, phi_dec=ph)
    rep = plan.apply_ex(xd, adjoint=adj, theta_dec=th, phi_dec=ph, replay=True)
    torch.cuda.synchronize()
    a, b = rec.cpu().numpy(), rep.cpu().numpy()
    assert np.array_equal(a, b)
    kw = dict(parity=parity, rho=rho, L=L, kind=kind, floor_modes=floor)
    ref = (oracle.adjoint if adj else oracle.forward)(x, **kw)
    assert rel(a, ref, x) <= TOL
    first = oracle.phi_pass(x, **kw) if adj else oracle.theta_pass(x, **kw)
    th_ref = oracle.decisions(first if adj else x, parity=parity, kind=kind)[0]
    ph_ref = oracle.decisions(x if adj else first, parity=parity, kind=kind)[1]
    hyb = kind == 3
    assert np.array_equal(th.cpu().numpy()[hyb], th_ref[hyb])
    assert np.array_equal(ph.cpu().numpy()[hyb], ph_ref[hyb])
    plan.close()
