"""The theta pass as a circulant product on the FP64 matrix cores
(SPHFILT_THETA_MFMA), on grids with n_phi = 2 n_theta in {32, 64}.

On one extended theta line the filter is the circular convolution with the
inverse transform of the mask (Sec. II.A, theta filter), and the lines of a
shell share it, so the variant computes the same operator by another
summation: it must match the oracle to 1e-12 (forward, adjoint, theta pass
alone; in place and out of place; fused shells and two passes; every kind and
parity; identity shells mixed in) and the FFT variant to rounding.
"""
import numpy as np
import pytest

import oracle
from paper_2305_01537_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def make_case(n_theta, seed, F=6, R=7):
    rng = np.random.default_rng(seed)
    shape = (F, R, n_theta, 2 * n_theta)
    x = rng.standard_normal(shape)
    parity = rng.choice([1, -1], F).astype(np.int32)
    kind = np.array([0, 1, 2, 0, 1, 2][:F], dtype=np.int32)
    # a spread of cutoffs: the outer shells of the large-L fields are identity
    L = np.array([0.3, 0.9, 2.5, 6.0, 0.5, 1.7][:F])
    return x, parity, kind, L


@pytest.mark.parametrize("n_theta", [16, 32])
@pytest.mark.parametrize("fused", [True, False], ids=["fused", "two-pass"])
def test_mfma_theta_matches_oracle(n_theta, fused):
    import torch
    from paper_2305_01537_amd.filter import THETA_MFMA, Plan
    x, parity, kind, L = make_case(n_theta, seed=n_theta + (1 if fused else 0))
    F, R, T, P = x.shape
    plan = Plan(R, T, P, F, parity=parity, L=L, kind=kind)
    plan.set_fused(fused)
    plan.set_theta_variant(THETA_MFMA)
    assert plan.get_theta_variant() == THETA_MFMA
    st = plan.stats()
    assert 0 < st["theta_shells_active"] < F * R      # identity shells mixed in
    kw = dict(parity=parity, L=L, kind=kind)
    refs = {"forward": oracle.forward(x, **kw), "adjoint": oracle.adjoint(x, **kw),
            "theta": oracle.theta_pass(x, **kw)}
    calls = {"forward": plan.apply, "adjoint": plan.apply_adjoint, "theta": plan.apply_theta}
    for name, fn in calls.items():
        for inplace in (True, False):
            xd = torch.from_numpy(x).cuda()
            y = fn(xd, out=xd) if inplace else fn(xd)
            torch.cuda.synchronize()
            err = rel(y.cpu().numpy(), refs[name])
            print(f"[gpu] mfma N={2 * n_theta} fused={fused} {name} inplace={inplace} err {err:.2e}",
                  flush=True)
            assert err <= TOL, (name, inplace, err)
    plan.close()


@pytest.mark.parametrize("n_theta", [16, 32])
def test_mfma_equals_fft_to_rounding_and_hybrid_keeps_fft(n_theta):
    """Both variants on the same plan agree to rounding; a hybrid field in the
    same plan takes the FFT in both (the circulant needs one kind per shell)."""
    import torch
    from paper_2305_01537_amd.filter import THETA_FFT, THETA_MFMA, Plan
    x, parity, kind, L = make_case(n_theta, seed=5 * n_theta)
    kind = kind.copy()
    kind[4] = 3                                   # hybrid
    x[4, 2, :, : n_theta // 2] += 3.0             # a jump: some lines take the Gaussian
    F, R, T, P = x.shape
    plan = Plan(R, T, P, F, parity=parity, L=L, kind=kind)
    outs = {}
    for v in (THETA_FFT, THETA_MFMA):
        plan.set_theta_variant(v)
        outs[v] = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(outs[THETA_MFMA], outs[THETA_FFT]) <= 1e-14
    ref = oracle.forward(x, parity=parity, L=L, kind=kind)
    assert rel(outs[THETA_MFMA], ref) <= TOL
    plan.close()


def test_mfma_variant_rejected_on_other_grids():
    from paper_2305_01537_amd.filter import THETA_MFMA, Plan, SphfiltError
    for T, P in ((64, 128), (16, 64), (128, 256)):
        plan = Plan(2, T, P, 1)
        with pytest.raises(SphfiltError):
            plan.set_theta_variant(THETA_MFMA)
        with pytest.raises(SphfiltError):
            plan.set_theta_variant(7)
        plan.close()


@pytest.mark.parametrize("N", [32, 64])
def test_mfma_dense_short_line_grid_sampled_shells(N):
    """The dense short-line benchmark grid (24 fields, ~800 MB, every line
    filtered) in the launch shape the benchmark times for the variant (fused,
    in place): sampled whole shells against the oracle."""
    import torch
    from paper_2305_01537_amd.filter import THETA_MFMA, Plan
    F, T, P = 24, N // 2, N
    R = int(800e6 // (F * T * P * 8))
    g = torch.Generator(device="cuda").manual_seed(N)
    x = torch.randn((F, R, T, P), dtype=torch.float64, device="cuda", generator=g)
    parity = np.where(np.arange(F) % 3 == 2, -1, 1)
    plan = Plan(R, T, P, F, parity=parity, L=0.2, rho=np.ones(R))
    plan.set_theta_variant(THETA_MFMA)
    rng = np.random.default_rng(N)
    picks = [(0, 0), (F - 1, R - 1)] + [tuple(v) for v in zip(rng.integers(0, F, 6), rng.integers(0, R, 6))]
    before = {p: x[p[0], p[1]].cpu().numpy() for p in picks}
    for fused in (True, False):
        plan.set_fused(fused)
        y = plan.apply(x)
        torch.cuda.synchronize()
        for f, i in picks:
            want = oracle.forward(before[(f, i)][None, None], parity=parity[f:f + 1], rho=[1.0], L=0.2)
            assert rel(y[f, i].cpu().numpy()[None, None], want) <= TOL, (fused, f, i)
        del y
    plan.close()
