"""The autotuners: every schedule they can pick filters correctly, their
picks are recorded in (and restored from) the JSON cache, and the pick is
never slower than the untuned schedule by the tuner's own timing.

Batch schedule knobs: split, workgroups per CU, fused items, the theta
sub-tile width of each line length, meridian tiles per theta item and ring
groups per phi item.  Plan knobs: theta tile width, ring pairs per phi
workgroup, fused shells, the theta variant and the overlap mode.
"""
import json
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def patch_set(seed=17):
    """Patches of every power-of-two line length, with identity shells, odd
    parities, all plain kinds; two-pass and fusable grids."""
    rng = np.random.default_rng(seed)
    shapes = [(2, 5, 16, 32), (3, 4, 32, 64), (2, 3, 64, 128), (2, 3, 128, 256), (1, 4, 32, 128),
              (2, 2, 64, 256), (3, 6, 16, 64), (1, 2, 128, 128)]
    out = []
    for F, R, T, P in shapes:
        out.append(dict(n_fields=F, n_r=R, n_theta=T, n_phi=P,
                        parity=rng.choice([1, -1], F).astype(np.int32),
                        L=rng.choice([0.3, 0.8, 3.0], F), kind=rng.choice([0, 1, 2], F).astype(np.int32),
                        rho=0.5 + np.arange(R) * rng.uniform(0.5, 2.0),
                        x=rng.standard_normal((F, R, T, P))))
    return out


def run(torch, batch, patches, adjoint=False):
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    outs = batch.apply(xs, adjoint=adjoint, check=True)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def schedules():
    """Each knob away from the default alone, and a few combinations."""
    base = dict(split=0, workgroups_per_cu=-1, fused=True, theta_tiles=1, phi_groups=1, theta_cols={})
    out = [base]
    for k, vals in (("split", (1, 2)), ("workgroups_per_cu", (1, 0)), ("fused", (False,)),
                    ("theta_tiles", (2, 4, 8)), ("phi_groups", (2, 4, 8))):
        for v in vals:
            out.append(dict(base, **{k: v}))
    for n in (32, 64, 128, 256):
        for w in (4, 8, 16, 32, 64):
            out.append(dict(base, theta_cols={n: w}))
    out.append(dict(split=1, workgroups_per_cu=0, fused=False, theta_tiles=4, phi_groups=2,
                    theta_cols={32: 4, 64: 8, 128: 16, 256: 8}))
    out.append(dict(split=2, workgroups_per_cu=-1, fused=True, theta_tiles=2, phi_groups=8,
                    theta_cols={64: 4, 256: 16}))
    out.append(dict(split=0, workgroups_per_cu=0, fused=False, theta_tiles=8, phi_groups=4,
                    theta_cols={128: 4, 32: 8}))
    return out


@pytest.mark.parametrize("adjoint", [False, True], ids=["forward", "adjoint"])
def test_every_batch_schedule_matches_the_oracle(adjoint):
    import torch
    from paper_2305_01537_amd.filter import Batch
    patches = patch_set()
    fn = oracle.adjoint if adjoint else oracle.forward
    refs = [fn(p["x"], parity=p["parity"], rho=p["rho"], L=p["L"], kind=p["kind"]) for p in patches]
    batch = Batch(patches)
    base = None
    n_run = 0
    for sch in schedules():
        try:
            batch.set_schedule_ex(**sch)
        except Exception:
            # a tile width no patch of that line length takes is rejected or falls back
            continue
        got = run(torch, batch, patches, adjoint)
        n_run += 1
        for k, (g, r) in enumerate(zip(got, refs)):
            assert rel(g, r) <= TOL, (sch, k, rel(g, r))
        if base is None:
            base = got
        for g, b in zip(got, base):
            assert rel(g, b) <= 1e-14, sch
    assert n_run >= 20
    batch.close()


def test_batch_tuner_records_and_restores_every_knob(tmp_path):
    import torch
    from paper_2305_01537_amd.filter import Batch
    patches = patch_set(seed=23)
    cache = tmp_path / "tune.json"
    batch = Batch(patches, tune_cache=str(cache))
    sch = batch.get_schedule()
    assert 0 < sch["tuned_us"] <= sch["default_us"]
    entries = json.loads(cache.read_text())["entries"]
    assert len(entries) == 1
    e = entries[0]
    for key in ("split", "wpc", "fused", "theta_tiles", "phi_groups", "theta_cols", "us", "default_us"):
        assert key in e, key
    assert e["what"] == "batch"
    # a second batch of the same patches takes the schedule from the cache
    again = Batch(patches, tune_cache=str(cache))
    s2 = again.get_schedule()
    for key in ("split", "workgroups_per_cu", "fused", "theta_tiles", "phi_groups", "theta_cols"):
        assert s2[key] == sch[key], key
    got = run(torch, again, patches)
    for p, g in zip(patches, got):
        ref = oracle.forward(p["x"], parity=p["parity"], rho=p["rho"], L=p["L"], kind=p["kind"])
        assert rel(g, ref) <= TOL
    batch.close()
    again.close()


def test_tune_cache_from_the_environment(tmp_path, monkeypatch):
    """A NULL cache path means the file named by SPHFILT_TUNE_CACHE."""
    from paper_2305_01537_amd.filter import Batch
    cache = tmp_path / "env_tune.json"
    monkeypatch.setenv("SPHFILT_TUNE_CACHE", str(cache))
    batch = Batch(patch_set(seed=3)[:3])
    assert cache.exists() and batch.get_schedule()["tuned_us"] > 0
    batch.close()
    monkeypatch.delenv("SPHFILT_TUNE_CACHE")
    untuned = Batch(patch_set(seed=3)[:3])
    assert untuned.get_schedule()["tuned_us"] < 0
    untuned.close()


@pytest.mark.parametrize("shape", [(3, 6, 32, 64), (2, 5, 64, 128), (2, 4, 128, 256), (4, 9, 16, 32)])
def test_plan_tuner_pick_and_cache(tmp_path, shape):
    import torch
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = shape
    rng = np.random.default_rng(T)
    x = rng.standard_normal(shape)
    parity = rng.choice([1, -1], F)
    L = rng.choice([0.4, 3.0], F)
    cache = tmp_path / "plan_tune.json"
    plan = Plan(R, T, P, F, parity=parity, L=L)
    times = plan.tune(str(cache))
    assert 0 < times["tuned_us"] <= times["default_us"]
    picked = (plan.get_schedule(), plan.get_fused(), plan.get_theta_variant(), plan.get_overlap())
    y = plan.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert rel(y, oracle.forward(x, parity=parity, L=L)) <= TOL
    e = json.loads(cache.read_text())["entries"][0]
    assert e["what"] == "plan" and "theta_cols" in e and "phi_lines" in e
    other = Plan(R, T, P, F, parity=parity, L=L)
    other.tune(str(cache))                       # restored from the cache, not re-timed
    assert (other.get_schedule(), other.get_fused(), other.get_theta_variant(),
            other.get_overlap()) == picked
    plan.close()
    other.close()
