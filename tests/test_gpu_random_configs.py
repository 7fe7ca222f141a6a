"""Seeded sweep over plan configurations, against the oracle.

Each case draws a grid (2 n_theta and n_phi among the supported line lengths,
radix-3 and radix-5 ones included, so grids with fused shells, with overlapped passes and
plain ones all occur),
per-field kinds (exponential, Gaussian, sharp, hybrid) and parities, cut-off
scales over two decades, a radius table (uniform, stretched or None), a floor,
the call (forward or adjoint, in place or out of place) and the schedule
(fused shells and overlap on or off, theta tile and ring pairs per
workgroup).  The result must match the oracle to 1e-12 relative max-norm, and
the same call with the plain two-pass schedule to 1e-14.
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


def run(torch, plan, x, call):
    xd = torch.from_numpy(x).cuda()
    fn = plan.apply_adjoint if call["adjoint"] else plan.apply
    y = fn(xd, out=xd) if call["inplace"] else fn(xd)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("seed", range(48))
def test_random_configuration(torch_gpu, seed):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    x, parity, kind, L, rho, floor, call = draw(seed)
    F, R, T, P = x.shape
    print(f"[gpu] case {seed}: {x.shape} kind {kind.tolist()} {call}", flush=True)
    plan = Plan(R, T, P, F, parity=parity, L=L, rho=rho, kind=kind, floor_modes=floor)
    plan.set_fused(call["fused"])
    plan.set_overlap(call["overlap"])
    got = run(torch, plan, x, call)
    ref_fn = oracle.adjoint if call["adjoint"] else oracle.forward
    ref = ref_fn(x, parity=parity, rho=rho, L=L, kind=kind, floor_modes=floor)
    assert rel(got, ref) <= TOL, (seed, rel(got, ref))
    # the plain schedule: both passes on the caller's stream, no fused shells
    plan.set_fused(False)
    plan.set_overlap(0)
    plain = run(torch, plan, x, call)
    assert rel(got, plain) <= 1e-14, (seed, rel(got, plain))
    plan.close()
