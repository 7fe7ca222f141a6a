"""Differentiation on the chain workload: 24 fields on 128 x 64 x 128, K = 8
applications of y <- tanh(F y), loss sum (y_K - t)^2.

Checks: the dot-product test <F x, y> = <x, F^T y>, the autograd gradient
against central finite differences (h = 1e-6) on 100 seeded entries, and
checkpointed against plain gradients.
"""
import numpy as np
import pytest

from paper_2305_01537_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_01537_amd.filter import Plan
    w = synth.workload("chain")
    F, R, T, P = w.shape
    plans = {L: Plan(R, T, P, F, parity=w.parity, L=L, rho=w.rho) for L in (3.0, 0.2)}
    return torch, w, plans


def _dot(a, b):
    # extended-precision accumulation of an FP64 dot product
    return np.sum(a.astype(np.longdouble) * b.astype(np.longdouble))


@pytest.mark.parametrize("L", [3.0, 0.2])
def test_dot_product(env, L):
    torch, w, plans = env
    plan = plans[L]
    rng = np.random.default_rng(51)
    x = rng.standard_normal(w.shape)
    y = rng.standard_normal(w.shape)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    Fx = plan.apply(xd).cpu().numpy()
    Fty = plan.apply_adjoint(yd).cpu().numpy()
    lhs, rhs = _dot(Fx, y), _dot(x, Fty)
    err = float(abs(lhs - rhs) / (np.linalg.norm(Fx) * np.linalg.norm(y)))
    print(f"[gpu] dot test L={L}: {err:.2e}", flush=True)
    assert err <= 1e-13


def test_autograd_uses_the_adjoint(env):
    torch, w, plans = env
    from paper_2305_01537_amd.autograd import sph_filter
    plan = plans[0.2]
    rng = np.random.default_rng(52)
    x = torch.from_numpy(rng.standard_normal(w.shape)).cuda().requires_grad_(True)
    g = torch.from_numpy(rng.standard_normal(w.shape)).cuda()
    y = sph_filter(x, plan)
    y.backward(g)
    ref = plan.apply_adjoint(g)
    assert torch.equal(x.grad, ref)


def test_autograd_takes_views_that_start_mid_way(env):
    # the library wants 16-byte aligned fields; the autograd layer copies a
    # view that starts at an odd double (input and incoming gradient alike)
    torch, w, plans = env
    from paper_2305_01537_amd.autograd import sph_filter
    plan = plans[3.0]
    n = int(np.prod(w.shape))
    rng = np.random.default_rng(53)
    xb = torch.from_numpy(rng.standard_normal(n + 1)).cuda().requires_grad_(True)
    gb = torch.from_numpy(rng.standard_normal(n + 1)).cuda()
    x, g = xb[1:].view(w.shape), gb[1:].view(w.shape)
    assert x.data_ptr() % 16 == 8 and g.data_ptr() % 16 == 8
    y = sph_filter(x, plan)
    y.backward(g)
    assert torch.equal(y.detach(), plan.apply(x.detach().clone()))
    assert torch.equal(xb.grad[1:].view(w.shape), plan.apply_adjoint(g.clone()))
    assert float(xb.grad[0]) == 0.0


def _loss_and_grad(torch, x, t, plan, K, checkpoint):
    from paper_2305_01537_amd.autograd import filter_chain
    xv = x.clone().requires_grad_(True)
    y = filter_chain(xv, plan, K, checkpoint=checkpoint)
    loss = ((y - t) ** 2).sum()
    loss.backward()
    return loss.detach(), xv.grad


def test_gradient_finite_differences_and_checkpointing(env):
    torch, w, plans = env
    from paper_2305_01537_amd.autograd import filter_chain
    plan = plans[3.0]
    K = 8
    x = torch.from_numpy(w.x).cuda()
    t = torch.from_numpy(w.target).cuda()
    _, g_ck = _loss_and_grad(torch, x, t, plan, K, checkpoint=True)
    _, g_plain = _loss_and_grad(torch, x, t, plan, K, checkpoint=False)
    rel_ck = float((g_ck - g_plain).abs().max() / g_plain.abs().max())
    print(f"[gpu] checkpointed vs plain gradient: {rel_ck:.2e}", flush=True)
    assert rel_ck <= 1e-15

    rng = np.random.default_rng(5)
    idx = rng.choice(x.numel(), size=100, replace=False)
    h = 1e-6
    # Floating-point noise of the difference quotient: y+ and y- of the
    # perturbed shell (n_theta * n_phi points) each carry ~eps relative
    # rounding, so L(x+h) - L(x-h) is known to about
    # eps * sqrt(points) * rms(y+ + y- - 2t), i.e. sigma below after / 2h.
    T, P = w.shape[2], w.shape[3]
    with torch.no_grad():
        y0 = filter_chain(x, plan, K, checkpoint=False)
        rms = float(torch.sqrt(torch.mean((2 * y0 - 2 * t) ** 2)))
    sigma = np.finfo(np.float64).eps * np.sqrt(T * P) * rms / (2 * h)
    rel_errs, excess = [], 0.0
    with torch.no_grad():
        for k in idx:
            xp = x.clone().view(-1)
            xm = x.clone().view(-1)
            xp[k] += h
            xm[k] -= h
            yp = filter_chain(xp.view(x.shape), plan, K, checkpoint=False)
            ym = filter_chain(xm.view(x.shape), plan, K, checkpoint=False)
            # L(x+h) - L(x-h) = sum (y+ - y-)(y+ + y- - 2t), summed without cancellation
            dl = float(((yp - ym) * (yp + ym - 2 * t)).sum())
            fd = dl / (2 * h)
            ad = float(g_ck.view(-1)[k])
            rel_errs.append(abs(fd - ad) / max(abs(ad), 1e-300))
            excess = max(excess, abs(fd - ad) / (1e-6 * abs(ad) + 4 * sigma))
    print(f"[gpu] finite differences over 100 entries: median rel err {np.median(rel_errs):.2e}, "
          f"worst {max(rel_errs):.2e}, noise floor {sigma:.1e}, worst err/(1e-6|g| + 4 sigma) {excess:.2f}",
          flush=True)
    assert np.median(rel_errs) <= 1e-7
    assert excess <= 1.0


@pytest.mark.parametrize("shape", [(4, 10, 48, 96), (3, 8, 80, 160), (2, 6, 96, 192)])
def test_dot_product_and_gradient_on_mixed_radix_grids(env, shape):
    """Lines with a radix-3 or radix-5 stage: the adjoint call is the transpose
    of the forward one (dot test), and autograd's gradient through the filter
    is that adjoint, bit for bit."""
    torch = env[0]
    from paper_2305_01537_amd.autograd import sph_filter
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = shape
    rng = np.random.default_rng(T + P)
    parity = np.where(np.arange(F) % 2 == 0, 1, -1).astype(np.int32)
    kind = np.array([0, 1, 2, 0][:F], dtype=np.int32)
    plan = Plan(R, T, P, F, parity=parity, L=0.5, kind=kind)
    x = rng.standard_normal(shape)
    y = rng.standard_normal(shape)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    Fx = plan.apply(xd).cpu().numpy()
    Fty = plan.apply_adjoint(yd).cpu().numpy()
    err = float(abs(_dot(Fx, y) - _dot(x, Fty)) / (np.linalg.norm(Fx) * np.linalg.norm(y)))
    print(f"[gpu] dot test {shape}: {err:.2e}", flush=True)
    assert err <= 1e-13
    xv = xd.clone().requires_grad_(True)
    sph_filter(xv, plan).backward(yd)
    assert torch.equal(xv.grad, plan.apply_adjoint(yd))
    plan.close()
