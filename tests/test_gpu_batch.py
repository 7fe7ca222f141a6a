"""Batched filter: many uneven patches in one graph-replayed launch.

Each patch must come out exactly as its own plan makes it (bit for bit: the
same per-line arithmetic), for every schedule (one kernel with per-shell
dependencies or two kernels; persistent or one workgroup per item), in place
and out of place, forward and adjoint; graph replays must see fresh data; and
the plans themselves are checked against the oracle elsewhere, here again on
small patches.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2305_01537_amd import synth

pytestmark = pytest.mark.gpu


def mixed_patches(seed=41):
    """Uneven patches, including theta-line and ring lengths that differ."""
    rng = np.random.default_rng(seed)
    shapes = [(3, 5, 16, 32), (2, 9, 16, 64), (4, 7, 32, 64), (1, 3, 32, 32), (5, 6, 64, 128),
              (2, 4, 64, 256), (3, 4, 128, 256), (2, 3, 128, 64), (6, 11, 16, 256), (1, 1, 64, 32),
              (7, 12, 32, 128), (2, 2, 128, 128)]
    out = []
    for F, R, T, P in shapes:
        out.append(dict(n_fields=F, n_r=R, n_theta=T, n_phi=P,
                        parity=rng.choice([1, -1], F).astype(np.int32),
                        L=rng.choice([0.3, 0.8, 3.0, 12.0], F),
                        kind=rng.choice([0, 0, 1, 2], F).astype(np.int32),
                        rho=0.5 + np.arange(R) * rng.uniform(0.5, 2.0),
                        x=rng.standard_normal((F, R, T, P))))
    return out


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def plan_outputs(torch, patches, adjoint, inplace, fused=False):
    from paper_2305_01537_amd.filter import Plan
    res = []
    for p in patches:
        F, R, T, P = p["x"].shape
        plan = Plan(R, T, P, F, parity=p["parity"], L=p["L"], rho=p["rho"], kind=p["kind"])
        plan.set_fused(fused)
        x = torch.from_numpy(p["x"]).cuda()
        fn = plan.apply_adjoint if adjoint else plan.apply
        y = fn(x, out=x) if inplace else fn(x)
        torch.cuda.synchronize()
        res.append(y.cpu().numpy())
        plan.close()
    return res


def same(a, b):
    return bool(np.array_equal(a, b))


def close(a, b, tol=1e-14):
    """Equal to rounding: a fused batch and fused plans run the same worker in
    different kernels (multiply-adds contracted differently)."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) <= tol


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("inplace", [True, False])
def test_batch_equals_plans_every_schedule(torch_gpu, adjoint, inplace):
    """Two-pass batch against two-pass plans: the same workers on the same
    lines, so bitwise equal in every schedule."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    patches = mixed_patches()
    ref = plan_outputs(torch, patches, adjoint, inplace)
    batch = Batch(patches)
    batch.set_fused(False)
    for split in (0, 1, 2):
        for wpc in (-1, 1, 0):
            batch.set_schedule(split, wpc)
            xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
            print(f"[gpu] batch adjoint={adjoint} inplace={inplace} split={split} wpc={wpc}", flush=True)
            ys = batch.apply(xs, outs=xs if inplace else None, adjoint=adjoint)
            torch.cuda.synchronize()
            assert batch.status() == 0
            for i, (y, r) in enumerate(zip(ys, ref)):
                ok = same(y.cpu().numpy(), r)
                assert ok, (split, wpc, i)
    batch.close()


@pytest.mark.parametrize("split,wpc,inplace", [(0, -1, False), (2, -1, True), (2, 1, True)])
def test_batch_graph_replays_see_fresh_data(torch_gpu, split, wpc, inplace):
    """Each call replays the cached graph (split = 2 in place: with its parallel
    branch) on new values written into the same buffers."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    patches = mixed_patches(43)
    batch = Batch(patches)
    batch.set_schedule(split, wpc)
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    outs = xs if inplace else [torch.empty_like(x) for x in xs]
    rng = np.random.default_rng(44)
    for rep in range(4):
        # new values in the same buffers between replays, with eager work and syncs in between
        for p, x in zip(patches, xs):
            p["x"] = rng.standard_normal(p["x"].shape)
            x.copy_(torch.from_numpy(p["x"]))
        torch.cuda.synchronize()
        print(f"[gpu] replay split={split} wpc={wpc} inplace={inplace} rep={rep}", flush=True)
        batch.apply(xs, outs=outs)
        torch.cuda.synchronize()
        # fused plans as the reference (the batch fuses by default): equal to
        # rounding, while a replay on stale data would be off by O(1)
        ref = plan_outputs(torch, patches, False, inplace, fused=True)
        for i, (y, r) in enumerate(zip(outs, ref)):
            assert close(y.cpu().numpy(), r), (rep, i)
    assert batch.status() == 0


def test_batch_small_patches_against_oracle(torch_gpu):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    patches = mixed_patches(45)[:5]
    batch = Batch(patches)
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    ys = batch.apply(xs)
    ya = batch.apply(xs, adjoint=True)
    torch.cuda.synchronize()
    for p, y, a in zip(patches, ys, ya):
        kw = dict(parity=p["parity"], rho=p["rho"], L=p["L"], kind=p["kind"])
        ref = oracle.forward(p["x"], **kw)
        refa = oracle.adjoint(p["x"], **kw)
        assert np.abs(y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(a.cpu().numpy() - refa).max() <= 1e-12 * np.abs(refa).max()


def test_batch_tuner_and_cache(torch_gpu, tmp_path):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    patches = mixed_patches(46)
    cache = tmp_path / "tune.json"
    b1 = Batch(patches, tune_cache=str(cache))
    s1 = b1.get_schedule()
    assert s1["tuned_us"] > 0
    data = json.loads(cache.read_text())
    assert len(data["entries"]) == 1 and data["entries"][0]["split"] == s1["split"]
    fz = data["entries"][0]["fused"]          # the tuner times fused items on and off
    assert fz in (0, 1) and b1.get_fused()[0] == bool(fz)
    b2 = Batch(patches, tune_cache=str(cache))       # cache hit: no tuning
    s2 = b2.get_schedule()
    assert s2["split"] == s1["split"] and s2["workgroups_per_cu"] == s1["workgroups_per_cu"]
    # the recorded times come back with the schedule
    assert abs(s2["tuned_us"] - s1["tuned_us"]) <= 1e-6 * s1["tuned_us"]
    assert b2.get_fused()[0] == bool(fz)
    # another patch set adds a second entry
    b3 = Batch(patches[:4], tune_cache=str(cache))
    assert len(json.loads(cache.read_text())["entries"]) == 2
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    ref = plan_outputs(torch, patches, False, False, fused=bool(fz))
    for y, r in zip(b2.apply(xs), ref):
        assert close(y.cpu().numpy(), r)
    for b in (b1, b2, b3):
        b.close()


def test_batch_schedule_values(torch_gpu):
    from paper_2305_01537_amd.filter import Batch, SphfiltError
    batch = Batch(mixed_patches()[:3])
    for split in (0, 1, 2):
        batch.set_schedule(split, -1)
        assert batch.get_schedule()["split"] == split
    with pytest.raises(SphfiltError):
        batch.set_schedule(3, -1)
    with pytest.raises(SphfiltError):
        batch.set_schedule(0, -2)
    # 0 selects the most persistent workgroups per compute unit that fit; one
    # more than that is rejected
    batch.set_schedule(0, 0)
    most = batch.get_schedule()["workgroups_per_cu"]
    assert most >= 1
    batch.set_schedule(1, most)
    with pytest.raises(SphfiltError):
        batch.set_schedule(1, most + 1)
    batch.close()


def test_batch_rejects_overlaps(torch_gpu):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch, SphfiltError
    patches = mixed_patches()[:2]
    batch = Batch(patches)
    n0 = patches[0]["x"].size
    buf = torch.zeros(n0 + patches[1]["x"].size, dtype=torch.float64, device="cuda")
    a = buf[:n0].view(patches[0]["x"].shape)
    b = buf[n0 - 8: n0 - 8 + patches[1]["x"].size].view(patches[1]["x"].shape)   # overlaps a
    with pytest.raises(SphfiltError):
        batch.apply([a, torch.zeros_like(b)], outs=[a, b])


def test_batch_patches_workload(torch_gpu):
    """The 64-patch workload (N_theta in 16..128, N_phi = 2 N_theta, 1..24 fields)."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    pts = synth.patches()
    patches = [dict(n_fields=p.n_fields, n_r=p.n_r, n_theta=p.n_theta, n_phi=p.n_phi, parity=p.parity,
                    L=p.L, rho=p.rho, kind=p.kind, x=p.x) for p in pts]
    print(f"[gpu] patches workload: {sum(p['x'].size for p in patches)} points", flush=True)
    ref = plan_outputs(torch, patches, False, True, fused=True)
    batch = Batch(patches)
    xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
    batch.apply(xs, outs=xs)
    torch.cuda.synchronize()
    assert batch.status() == 0
    for i, (y, r) in enumerate(zip(xs, ref)):
        assert close(y.cpu().numpy(), r), i


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("inplace", [True, False])
def test_fused_batch_matches_fused_plans_every_schedule(torch_gpu, adjoint, inplace):
    """With fused items (patches with n_phi = 2 n_theta <= 128): the batch and
    fused plans run the same shell worker in different kernels, so they agree
    to rounding; in place equals out of place bitwise across schedules."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Batch
    patches = mixed_patches()
    ref = plan_outputs(torch, patches, adjoint, inplace, fused=True)
    batch = Batch(patches)
    enabled, n_fused = batch.get_fused()
    st = batch.stats()
    assert enabled and n_fused == st["shells_fused"] > 0
    assert st["bytes_fused_inplace"] < st["bytes_forward_inplace"]
    first = None
    for split in (0, 1, 2):
        for wpc in (-1, 1, 0):
            batch.set_schedule(split, wpc)
            xs = [torch.from_numpy(p["x"]).cuda() for p in patches]
            print(f"[gpu] fused batch adjoint={adjoint} inplace={inplace} split={split} wpc={wpc}", flush=True)
            ys = batch.apply(xs, outs=xs if inplace else None, adjoint=adjoint)
            torch.cuda.synchronize()
            assert batch.status() == 0
            got = [y.cpu().numpy() for y in ys]
            for i, (g, r) in enumerate(zip(got, ref)):
                assert close(g, r), (split, wpc, i)
            if first is None:
                first = got
            for g, f in zip(got, first):
                assert np.array_equal(g, f), (split, wpc)
    batch.set_fused(False)
    assert batch.get_fused() == (False, 0)
    assert batch.stats()["bytes_fused_inplace"] == batch.stats()["bytes_forward_inplace"]
    batch.close()
