"""Buffers past 32-bit offsets.

One field of 66,000 shells of 128 x 256 (17.3 GB): byte offsets pass 2^32 at
shell 16,384 and point offsets pass 2^31 at shell 65,536.  A plan filters it
in place (forward) and out of place (adjoint), and a batch with a small second
patch filters it in place; shells on both sides of both boundaries, with the
theta pass active and idle, must match the oracle.  The radius table cycles
so that shells far out still filter.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
TOL = 1e-12
R, T, P = 66000, 128, 256
SAMPLE = [0, 16383, 16384, 16385, 65535, 65536, 65537, 65999]
L = np.array([3.0])
PARITY = np.array([-1], dtype=np.int32)


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    rho = 0.5 + (np.arange(R) % 64) * 0.5
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn((1, R, T, P), dtype=torch.float64, device="cuda", generator=g)
    torch.cuda.synchronize()
    yield torch, x, rho
    del x
    torch.cuda.empty_cache()


def sampled(t):
    return t[:, SAMPLE].cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check(got, x0, rho, fn):
    ref = fn(x0, parity=PARITY, rho=rho[SAMPLE], L=L)
    for k, i in enumerate(SAMPLE):
        assert rel(got[:, k], ref[:, k]) <= TOL, (i, rel(got[:, k], ref[:, k]))


def test_plan_past_32_bit_offsets(big):
    torch, x, rho = big
    from paper_2305_01537_amd.filter import Plan
    print(f"[gpu] large plan {tuple(x.shape)}", flush=True)
    x0 = sampled(x)
    plan = Plan(R, T, P, 1, parity=PARITY, L=L, rho=rho)
    st = plan.stats()
    assert 0 < st["theta_shells_active"] < R
    y = plan.apply_adjoint(x)                   # out of place: x unchanged
    torch.cuda.synchronize()
    check(sampled(y), x0, rho, oracle.adjoint)
    del y
    torch.cuda.empty_cache()
    plan.apply(x, out=x)                        # in place
    torch.cuda.synchronize()
    check(sampled(x), x0, rho, oracle.forward)
    plan.close()


def test_batch_past_32_bit_offsets(big):
    torch, x, rho = big
    from paper_2305_01537_amd.filter import Batch
    print(f"[gpu] large batch {tuple(x.shape)} + (2, 3, 32, 64)", flush=True)
    x0 = sampled(x)
    rng = np.random.default_rng(8)
    small = dict(n_fields=2, n_r=3, n_theta=32, n_phi=64, parity=np.array([1, -1], dtype=np.int32),
                 L=np.array([0.7, 2.0]), rho=None)
    xs0 = rng.standard_normal((2, 3, 32, 64))
    xs = torch.from_numpy(xs0).cuda()
    batch = Batch([dict(n_fields=1, n_r=R, n_theta=T, n_phi=P, parity=PARITY, L=L, rho=rho), small])
    batch.apply([x, xs], outs=[x, xs])
    torch.cuda.synchronize()
    assert batch.status() == 0
    check(sampled(x), x0, rho, oracle.forward)
    ref = oracle.forward(xs0, parity=small["parity"], L=small["L"])
    assert rel(xs.cpu().numpy(), ref) <= TOL
    batch.close()
