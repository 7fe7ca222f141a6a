"""bench.py's CPU context figure with library FFTs (cpu_fft_forward) computes
the same filter as the oracle (exponential kind, both parities, uniform and
stretched radii): a check of the benchmark's baseline, not of the GPU path."""
import numpy as np
import pytest

import bench
import oracle


@pytest.mark.parametrize("T,P,rho", [(8, 16, None), (16, 32, "stretched"), (12, 48, None), (32, 64, "stretched")])
def test_cpu_fft_forward_matches_the_oracle(T, P, rho):
    rng = np.random.default_rng(T * 100 + P)
    F, R = 3, 4
    x = rng.standard_normal((F, R, T, P))
    parity = np.array([1, -1, 1], dtype=np.int32)
    L = np.array([0.4, 1.3, 3.0])
    r = 0.5 + np.arange(R) if rho is None else np.cumsum(rng.uniform(0.3, 4.0, R))
    got = bench.cpu_fft_forward(x, parity, r, L, 2)
    want = oracle.forward(x, parity=parity, rho=r, L=L)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
