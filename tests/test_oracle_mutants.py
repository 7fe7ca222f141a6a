"""The pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle's C source (in a temporary
directory, on the CPU), builds it, and runs the pins of test_oracle_pins.py
against the mutant.  At least one pin must fail for every mutant; otherwise
the pins would not be strong enough to trust the oracle.
"""
import importlib.util
import os
import subprocess

import numpy as np
import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sphfilt_oracle.c")
WRAPPER = os.path.join(ROOT, "oracle", "oracle.py")

MUTANTS = {
    "extension sign dropped": ("g[n] = s * X[", "g[n] = X["),
    "extension not reversed": ("g[n] = s * X[(int64_t)(N - 1 - n) * n_phi", "g[n] = s * X[(int64_t)(n - n_theta) * n_phi"),
    "extension without the half-turn in phi": ("* n_phi + k + half];\n}", "* n_phi + k];\n}"),
    "write-back sign dropped": ("k + half] = s * o[n]", "k + half] = o[n]"),
    "passes swapped in forward": (
        "int rc = orc_theta_pass(in, tmp, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,\n"
        "                            floor_modes, &a);\n"
        "    if (!rc)\n"
        "        rc = orc_phi_pass(tmp, out,",
        "int rc = orc_phi_pass(in, tmp, n_fields, n_r, n_theta, n_phi, parity, rho, L, kind,\n"
        "                            floor_modes, &a);\n"
        "    if (!rc)\n"
        "        rc = orc_theta_pass(tmp, out,"),
    "mask on signed index": ("orc_mask(kind, (double)qhat, c)", "orc_mask(kind, (double)q, c)"),
    "exp filter off by one": ("exp(-(qhat - c))", "exp(-(qhat - c + 1.0))"),
    "cutoff missing factor 2": ("double c = 2.0 * rho * L;", "double c = rho * L;"),
    "latitude not cell-centred": ("((double)jm + 0.5) * ORC_PI", "((double)jm + 1.0) * ORC_PI"),
    "inverse normalisation": ("out[n] = re / (double)N;", "out[n] = re / (double)(N - 1);"),
    "conjugated forward transform": ("im -= g[n] * st[m];", "im += g[n] * st[m];"),
    "sharp mask drops the edge mode": ("return qhat <= c ? 1.0 : 0.0;", "return qhat < c ? 1.0 : 0.0;"),
    "gaussian constant": ("exp(log(0.9) * u * u)", "exp(log(0.8) * u * u)"),
    "floor ignored": ("return c > floor_modes ? c : floor_modes;\n}\n\n/* sin", "return c;\n}\n\n/* sin"),
    "phi cutoff without sin(theta)": ("double c = 2.0 * rho * orc_sin_theta(j, n_theta) * L;", "double c = 2.0 * rho * L;"),
    "detector never fires": ("if (sigma >= orc_det_threshold) return 1;", "if (sigma > 2.0) return 1;"),
    "detector not periodic": ("const double a = g[(n - 1 + N) % N], b = g[n], c = g[(n + 1) % N];",
                              "const double a = g[n > 0 ? n - 1 : 0], b = g[n], c = g[n + 1 < N ? n + 1 : N - 1];"),
    "detector ignores the centre weight": ("fabs(a - 2.0 * b + c)", "fabs(a - b + c)"),
    "mode index not reduced": ("int m = (int)(((int64_t)q * n) % N);\n            re += g[n]", "int m = (int)(((int64_t)q * n + n) % N);\n            re += g[n]"),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not unique"
    d = tmp_path / name.replace(" ", "_")
    d.mkdir()
    (d / "m.c").write_text(src.replace(old, new))
    so = d / "libm.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(so), str(d / "m.c"), "-lm"], check=True)
    spec = importlib.util.spec_from_file_location(f"orc_mut_{abs(hash(name))}", WRAPPER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.lib_path = str(so)
    mod._lib = None
    mod._load()
    return mod


def _pin_cases():
    P = pins
    return [
        lambda m: [P.test_p1_constant_even_parity(m, k) for k in (0, 1, 2)],
        lambda m: [P.test_p3_separable_eigenmodes(m, k, s, 16, 32) for k in (0, 1, 2) for s in (1, -1)],
        lambda m: P.test_p3_order_matters(m),
        lambda m: [P.test_p5_phi_rotation_equivariance(m, s) for s in (1, -1)],
        lambda m: [P.test_p5_equatorial_reflection(m, s) for s in (1, -1)],
        lambda m: P.test_p5_partner_meridian_own_line(m),
        lambda m: P.test_p7_dot_product(m),
        lambda m: P.test_p8_paper_constants(m),
        lambda m: P.test_p8_cutoff_depends_on_r_and_latitude(m),
        lambda m: [P.test_p10_library_fft_matches(m, k) for k in (0, 1, 2)],
        lambda m: P.test_p10_library_fft_matches_radix3_lengths(m, 24, 48),
        lambda m: P.test_p10_sharp_cutoff_on_a_mode_keeps_it(m),
        lambda m: P.test_hybrid_smooth_fields_take_the_exponential_filter(m),
        lambda m: P.test_hybrid_ring_with_a_jump_takes_the_gaussian(m),
        lambda m: P.test_hybrid_theta_decision_uses_the_extended_line(m),
        lambda m: P.test_hybrid_grid_scale_oscillation_is_detected(m),
        lambda m: P.test_hybrid_detector_is_periodic_and_has_a_threshold(m),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    mod = _build_mutant(tmp_path, name, old, new)
    failed = 0
    for case in _pin_cases():
        try:
            with np.errstate(all="ignore"):
                case(mod)
        except (AssertionError, ValueError):
            failed += 1
    assert failed > 0, f"no pin catches the mutant {name!r}"
