"""Seeded synthetic fields on an (r, theta, phi) grid.

This module only draws inputs; it contains none of the filter's arithmetic, so
both the GPU library's tests and the CPU oracle's tests take their inputs from
here.  Fields stand in for the evolved spacetime / GRMHD variables that the
paper filters (arXiv:2305.01537, Sec. II.A): smooth sums of real spherical
harmonics with a radial profile, plus white noise, with each field carrying an
axis parity sign (+1 scalars, +-1 vector/tensor components).

Grid: theta_j = (j + 1/2) pi / n_theta (cell centred, no point on a pole),
phi_k = 2 pi k / n_phi, rho_i = r_i / dr_min = i + 1/2 (uniform cell-centred
radial grid).

Named workloads (all FP64, layout [field][r][theta][phi], phi fastest):
  small     1 field, 16 x 32 x 64, even parity, harmonics l <= 8, noise 1e-3
  grmhd     24 fields, 128 x 64 x 128, 8 even scalars + 16 seeded-sign
            components, harmonics l <= 32 with angular power ~ l^-2, noise 1e-4
  share     the grmhd statistics on 24 fields, 256 x 128 x 256 (1.6 GB)
  patches   64 uneven patches (n_theta in {16,32,64,128}, n_phi = 2 n_theta,
            n_r in [8, 64], 1..24 fields each)
  chain     the grmhd shape and values, with a seeded N(0,1) target field
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray            # (F, n_r, n_theta, n_phi) float64
    parity: np.ndarray       # (F,) int32, +1 / -1
    rho: np.ndarray          # (n_r,) float64, r / dr_min
    L: np.ndarray            # (F,) float64, the cutoff scale cal-L
    kind: np.ndarray         # (F,) int32, 0 = exponential filter
    target: Optional[np.ndarray] = None

    @property
    def shape(self):
        return self.x.shape


SHAPES = {
    "small": (1, 16, 32, 64),
    "grmhd": (24, 128, 64, 128),
    "share": (24, 256, 128, 256),
    "chain": (24, 128, 64, 128),
}


def theta_grid(n_theta: int) -> np.ndarray:
    return (np.arange(n_theta, dtype=np.float64) + 0.5) * np.pi / n_theta


def phi_grid(n_phi: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n_phi, dtype=np.float64) / n_phi


def uniform_rho(n_r: int) -> np.ndarray:
    return np.arange(n_r, dtype=np.float64) + 0.5


def _legendre_table(lmax: int, theta: np.ndarray) -> np.ndarray:
    """P[l, m, j] = Y_l^m(theta_j, 0) (orthonormal, real for phi = 0)."""
    from scipy.special import sph_harm_y
    P = np.zeros((lmax + 1, lmax + 1, theta.size))
    for l in range(lmax + 1):
        for m in range(l + 1):
            P[l, m] = np.real(sph_harm_y(l, m, theta, 0.0))
    return P


def angular_sum(rng: np.random.Generator, lmax: int, theta: np.ndarray, phi: np.ndarray,
                std_of_l, P: Optional[np.ndarray] = None, max_m: Optional[int] = None) -> np.ndarray:
    """sum_{l <= lmax, |m| <= l} a_lm Y_lm(theta_j, phi_k), real Y_lm, a_lm ~ N(0, std(l)^2)."""
    if P is None:
        P = _legendre_table(lmax, theta)
    mm = lmax if max_m is None else min(lmax, max_m)
    l_idx = np.arange(lmax + 1)
    std = np.asarray([std_of_l(l) for l in l_idx])
    a_cos = rng.standard_normal((lmax + 1, lmax + 1)) * std[:, None]
    a_sin = rng.standard_normal((lmax + 1, lmax + 1)) * std[:, None]
    tri = l_idx[:, None] >= l_idx[None, :]          # m <= l
    a_cos *= tri
    a_sin *= tri
    m = np.arange(mm + 1)
    w = np.where(m == 0, 1.0, np.sqrt(2.0))
    C = np.einsum("lm,lmj->mj", a_cos[:, : mm + 1], P[:, : mm + 1]) * w[:, None]
    S = np.einsum("lm,lmj->mj", a_sin[:, : mm + 1], P[:, : mm + 1]) * w[:, None]
    S[0] = 0.0
    cos_mp = np.cos(np.outer(m, phi))
    sin_mp = np.sin(np.outer(m, phi))
    return C.T @ cos_mp + S.T @ sin_mp


def radial_profile(rng: np.random.Generator, n_r: int) -> np.ndarray:
    """R(rho_i) = sum_{q<4} b_q cos(q pi (i + 1/2) / n_r), b_q ~ N(0,1) / (1+q)^2."""
    b = rng.standard_normal(4) / (1.0 + np.arange(4)) ** 2
    s = (np.arange(n_r) + 0.5) / n_r
    return sum(b[q] * np.cos(q * np.pi * s) for q in range(4))


def parity_table(n_fields: int, rng: np.random.Generator, n_even: int = 8) -> np.ndarray:
    """First n_even fields are scalars (+1); the rest get seeded signs."""
    p = np.ones(n_fields, dtype=np.int32)
    if n_fields > n_even:
        p[n_even:] = rng.choice(np.array([1, -1], dtype=np.int32), n_fields - n_even)
    return p


def make_fields(shape, parity, lmax: int, std_of_l, noise: float, rng: np.random.Generator,
                max_m: Optional[int] = None) -> np.ndarray:
    F, n_r, n_theta, n_phi = shape
    theta, phi = theta_grid(n_theta), phi_grid(n_phi)
    P = _legendre_table(lmax, theta)
    x = np.empty(shape, dtype=np.float64)
    for f in range(F):
        A = angular_sum(rng, lmax, theta, phi, std_of_l, P, max_m)
        if parity[f] < 0:           # odd fields vanish on the axis like sin(theta)
            A = A * np.sin(theta)[:, None]
        R = radial_profile(rng, n_r)
        x[f] = R[:, None, None] * A[None, :, :]
        if noise > 0:
            x[f] += noise * rng.standard_normal((n_r, n_theta, n_phi))
    return x


def _grmhd_std(l):
    return 1.0 / (l + 1.0)


def workload(name: str, seed: Optional[int] = None, L: float = 3.0, shape=None) -> Workload:
    """Build one of the named workloads; `shape` overrides the grid for quick tests."""
    seeds = {"small": 1, "grmhd": 2, "share": 3, "patches": 4, "chain": 5}
    rng = np.random.default_rng(seeds[name] if seed is None else seed)
    shp = tuple(shape) if shape is not None else SHAPES[name]
    F, n_r, n_theta, n_phi = shp
    if name == "small":
        parity = np.ones(F, dtype=np.int32)
        x = make_fields(shp, parity, 8, lambda l: 1.0, 1e-3, rng)
    elif name in ("grmhd", "share", "chain"):
        parity = parity_table(F, rng)
        x = make_fields(shp, parity, min(32, n_theta - 1), _grmhd_std, 1e-4, rng)
    else:
        raise ValueError(f"unknown workload {name!r}")
    w = Workload(name, x, parity, uniform_rho(n_r), np.full(F, L), np.zeros(F, dtype=np.int32))
    if name == "chain":
        w.target = rng.standard_normal(shp)
    return w


@dataclasses.dataclass
class Patch:
    n_fields: int
    n_r: int
    n_theta: int
    n_phi: int
    parity: np.ndarray
    rho: np.ndarray
    L: np.ndarray
    kind: np.ndarray
    x: Optional[np.ndarray] = None


def patches(seed: int = 4, n_patches: int = 64, with_values: bool = True, L: float = 3.0,
            n_theta_choices=(16, 32, 64, 128), n_r_range=(8, 64), f_range=(1, 24)) -> List[Patch]:
    """Uneven spherical patches, each with its own shape, fields and parities."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_patches):
        n_theta = int(rng.choice(np.asarray(n_theta_choices)))
        n_r = int(rng.integers(n_r_range[0], n_r_range[1] + 1))
        F = int(rng.integers(f_range[0], f_range[1] + 1))
        parity = rng.choice(np.array([1, -1], dtype=np.int32), F).astype(np.int32)
        p = Patch(F, n_r, n_theta, 2 * n_theta, parity, uniform_rho(n_r), np.full(F, L),
                  np.zeros(F, dtype=np.int32))
        if with_values:
            p.x = make_fields((F, n_r, n_theta, 2 * n_theta), parity, min(32, n_theta - 1),
                              _grmhd_std, 1e-4, rng)
        out.append(p)
    return out
