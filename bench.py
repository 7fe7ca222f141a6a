#!/usr/bin/env python3
"""Benchmark of the double FFT filter on one MI355X.

One step = one forward double FFT filter (theta-pass then phi-pass) over the
production share: 24 FP64 fields on a 256 x 128 x 256 (r, theta, phi) grid,
with the paper's cutoff (cal-L = 3 on a uniform cell-centred radial grid),
applied in place -- the way an evolution code filters its state once per
Runge-Kutta substep, with the launch settings the plan's autotuner picks
(tile widths, ring pairs per workgroup, overlap of the rings that do not
depend on the theta pass on a second stream).  Inputs are seeded
synthetic fields already resident in HBM; four copies are rotated so no step
finds its data in the 256 MB Infinity Cache from the step before.

Prints ONE JSON line:
  value         filtered field-points per second (whole job, one GPU)
  roofline      the dominant kernel's algorithmic HBM bytes per launch over
                its average launch time (HIP events on the launch stream),
                against the 8 TB/s HBM3E peak
  cpu_baseline  the CPU oracle (direct DFTs) on a bounded sample of the same
                workload, on this host's cores (and on one thread)
  extra         adjoint/forward ratio, the forward on one stream, per-field
                launches, the dense-cutoff variant, the grmhd grid (fused
                shells), the 64-patch batch, dense short-line grids
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "share_paper_cutoff_counters.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2305_01537_amd", "csrc", f)
                  for f in ("kernels.hip", "kernels_theta.hip", "kernels_phi.hip", "line_filter.h",
                            "fft_core.h", "sphfilt_internal.h")]


def code_tokens(text):
    """C++ source with comments removed and whitespace collapsed: the code
    the counters were taken on (comment edits do not change it)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(read=None):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        if read is None:
            with open(f, encoding="utf-8") as fh:
                text = fh.read()
        else:
            text = read(f)
        h.update(code_tokens(text).encode())
    return h.hexdigest()[:16]


def counter_traffic(kernel, L):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size), or None
    when the kernels have changed since the counters were taken."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_hash") != kernel_source_hash() or L != 3.0:
        return None
    k = c.get("kernels", {}).get(kernel)
    return None if k is None else k["traffic_bytes"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # every timed loop is preceded by >= 30 ms of the same call on the GPU
    # (clock_warmup), whatever --warmup says
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--L", type=float, default=3.0, help="cutoff scale cal-L of every field")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="after the timed loops, run plain copies of the workload buffer "
                         "(reference for the HBM byte counters)")
    ap.add_argument("--patches-only", action="store_true",
                    help="time only the 64-patch batch and print its figures as JSON "
                         "(for profiling the batch kernel)")
    ap.add_argument("--batch-schedule", type=str, default=None,
                    help="with --patches-only: split,workgroups_per_cu,theta_tiles,phi_groups "
                         "set instead of the tuner's pick (for profiling one schedule)")
    ap.add_argument("--grmhd-only", action="store_true",
                    help="time only the grmhd grid, fused and two-pass, and print its figures "
                         "as JSON (for profiling the fused shell kernel)")
    ap.add_argument("--short-lines-only", action="store_true",
                    help="time only the dense short-line grids (n_phi = 32, 64, 128)")
    ap.add_argument("--mixed-radix-only", action="store_true",
                    help="time only the 96 x 192 and 80 x 160 grids (lines with a radix-3 or "
                         "radix-5 stage)")
    ap.add_argument("--hybrid-only", action="store_true",
                    help="time only the share with 8 hybrid fields and print its figures as JSON "
                         "(for profiling the hybrid-capable kernels)")
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="wall-time budget for sizing the oracle sample (sized from one shell's "
                         "time, which overestimates: the sample itself takes about 10 s on 16 "
                         "threads)")
    return ap.parse_args()


# GPU time of the same call run before every timed loop, whatever --warmup
# says: after host-side work the GPU takes ~10 ms of continuous load to reach
# its steady clock, and a loop timed from a cold start reads ~10 % slow.
CLOCK_WARMUP_MS = 30.0


def clock_warmup(torch, fn, bufs, stream, min_ms=CLOCK_WARMUP_MS):
    """Run fn in groups of 8 calls until the GPU has spent at least min_ms on
    them (HIP events on `stream`); returns the GPU time spent."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    spent, k = 0.0, 0
    while spent < min_ms and k < 100000:
        e0.record(stream)
        for _ in range(8):
            fn(bufs[k % len(bufs)])
            k += 1
        e1.record(stream)
        e1.synchronize()
        spent += e0.elapsed_time(e1)
    return spent


def time_loop(torch, fn, bufs, steps, warmup, stream, info=None):
    """Warm the clock (clock_warmup), run fn(buf) `warmup` times untimed, then
    `steps` times between HIP events recorded on `stream` (the stream the
    library launches on).  info, if given, receives the warm-up GPU time."""
    warm = clock_warmup(torch, fn, bufs, stream)
    if info is not None:
        info["clock_warmup_ms"] = warm
    for k in range(warmup):
        fn(bufs[k % len(bufs)])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for k in range(steps):
        fn(bufs[k % len(bufs)])
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps      # ms per call


def _median_rate(fn, points, reps):
    """Median over `reps` runs of points / wall time of fn()."""
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    ts.sort()
    return points / ts[len(ts) // 2], ts[len(ts) // 2]


def cpu_baseline(w, L, budget_s):
    """The oracle as it stands (direct DFTs, OpenMP over lines), timed on this
    host's cores.  `value`: the forward filter on whole shells of the share
    workload (one shell first to size the sample, then that many shells,
    field-major).  `legs`: the same oracle on the small and grmhd workloads,
    whole, forward and adjoint, median of 3 runs; the adjoint on the share
    sample; one thread on the small workload (whole) and on one field of the
    grmhd workload and of the share."""
    import numpy as np
    import oracle
    from paper_2305_01537_amd import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    F, R = w.shape[0], w.shape[1]
    t = time.perf_counter()
    oracle.forward(w.x[0:1, 0:1], parity=w.parity[0:1], rho=w.rho[0:1], L=L)
    one = time.perf_counter() - t
    n_sh = int(max(1, min(F * R, budget_s / max(one, 1e-6))))
    n_f = max(1, n_sh // R) if n_sh >= R else 1
    n_r = R if n_sh >= R else n_sh
    sub = np.ascontiguousarray(w.x[:n_f, :n_r])
    kw = dict(parity=w.parity[:n_f], rho=w.rho[:n_r], L=L)
    t = time.perf_counter()
    oracle.forward(sub, **kw)
    dt = time.perf_counter() - t
    t = time.perf_counter()
    oracle.adjoint(sub, **kw)
    dt_adj = time.perf_counter() - t
    legs = {"share_sample_adjoint": {"value": sub.size / dt_adj, "seconds": dt_adj}}
    singles = {}
    for name in ("small", "grmhd"):
        v = synth.workload(name)
        kw_v = dict(parity=v.parity, rho=v.rho, L=v.L)
        fwd, tf = _median_rate(lambda: oracle.forward(v.x, **kw_v), v.x.size, 3)
        adj, ta = _median_rate(lambda: oracle.adjoint(v.x, **kw_v), v.x.size, 3)
        legs[name] = {"shape": list(v.shape), "forward": fwd, "adjoint": adj,
                      "forward_s": tf, "adjoint_s": ta, "runs": 3, "stat": "median"}
    # one thread: the small workload whole, one field of grmhd, evenly spaced
    # shells of one field of the share (the same radial mix of theta-filtered
    # and theta-idle shells)
    prev = oracle.set_threads(1)
    v = synth.workload("small")
    singles["small"], _ = _median_rate(
        lambda: oracle.forward(v.x, parity=v.parity, rho=v.rho, L=v.L), v.x.size, 3)
    g = synth.workload("grmhd")
    g1 = np.ascontiguousarray(g.x[:1])
    singles["grmhd_field0"], _ = _median_rate(
        lambda: oracle.forward(g1, parity=g.parity[:1], rho=g.rho, L=g.L[:1]), g1.size, 1)
    n1 = int(max(1, min(R, budget_s / 4 / max(one * threads, 1e-6))))
    idx = np.unique(np.linspace(0, R - 1, n1).round().astype(int))
    sub1 = np.ascontiguousarray(w.x[:1, idx])
    t = time.perf_counter()
    oracle.forward(sub1, parity=w.parity[:1], rho=w.rho[idx], L=L)
    dt1 = time.perf_counter() - t
    singles["share_sample"] = sub1.size / dt1
    oracle.set_threads(prev)
    return {"value": sub.size / dt, "unit": "field-points/s", "cores": threads, "kind": "oracle",
            "sample": f"fields 0..{n_f - 1} x shells 0..{n_r - 1} of the share workload "
                      f"({sub.size} points, cal-L={L}), forward filter (theta then phi, "
                      f"direct DFTs), {dt:.1f} s",
            "host_cpu": host_cpu(),
            "legs": legs,
            "single_thread": {"unit": "field-points/s", "forward": singles,
                              "sample": f"small: whole (median of 3); grmhd: field 0 "
                                        f"({g1.size} points); share: field 0 x {len(idx)} "
                                        f"evenly spaced shells ({sub1.size} points, {dt1:.1f} s)"}}


def cpu_fft_forward(x, parity, rho, L, workers):
    """The forward filter (exponential kind) on the CPU with library FFTs
    (scipy.fft, pocketfft, `workers` threads): the paper's steps -- each
    meridian pair extended across the poles with the field's parity sign,
    transformed, damped above l_max = max(2, 2 rho L), transformed back; then
    each ring damped above m_max = max(2, 2 rho sin(theta) L) (Sec. II.A) --
    over every line, vectorised per field.  A context figure for the CPU
    with FFTs, as the paper filters; not the oracle (tests check the two
    agree)."""
    import numpy as np
    import scipy.fft as sf
    F, R, T, P = x.shape
    h = P // 2
    theta = (np.arange(T) + 0.5) * np.pi / T
    q = np.arange(T + 1, dtype=np.float64)            # rfft bins of a 2T line: |q| = q
    m = np.arange(h + 1, dtype=np.float64)            # rfft bins of a ring: |m| = m
    y = np.empty_like(x)
    for f in range(F):
        s = float(parity[f])
        ext = np.concatenate([x[f, :, :, :h], s * x[f, :, ::-1, h:]], axis=1)   # [R][2T][P/2]
        c = np.maximum(2.0, 2.0 * rho * L[f])[:, None, None]
        mask = np.where(q[None, :, None] <= c, 1.0, np.exp(-np.maximum(q[None, :, None] - c, 0.0)))
        g = sf.irfft(sf.rfft(ext, axis=1, workers=workers) * mask, n=2 * T, axis=1, workers=workers)
        z = np.empty_like(x[f])
        z[:, :, :h] = g[:, :T]
        z[:, :, h:] = s * g[:, T:][:, ::-1]
        cm = np.maximum(2.0, 2.0 * rho[:, None, None] * np.sin(theta)[None, :, None] * L[f])
        mask = np.where(m[None, None, :] <= cm, 1.0, np.exp(-np.maximum(m[None, None, :] - cm, 0.0)))
        y[f] = sf.irfft(sf.rfft(z, axis=2, workers=workers) * mask, n=P, axis=2, workers=workers)
    return y


def cpu_fft_baseline(w, L, budget_s):
    """cpu_fft_forward timed on whole fields of the share workload (one field
    first to size the sample to about budget_s seconds)."""
    import numpy as np
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    Lf = np.full(w.shape[0], float(L))
    t = time.perf_counter()
    cpu_fft_forward(w.x[:1], w.parity[:1], w.rho, Lf[:1], threads)
    one = time.perf_counter() - t
    n_f = int(max(1, min(w.shape[0], budget_s / max(one, 1e-6))))
    sub = w.x[:n_f]
    t = time.perf_counter()
    cpu_fft_forward(sub, w.parity[:n_f], w.rho, Lf[:n_f], threads)
    dt = time.perf_counter() - t
    return {"value": sub.size / dt, "unit": "field-points/s", "threads": threads,
            "kind": "scipy.fft (pocketfft) implementation of the same steps; context, not the oracle",
            "sample": f"fields 0..{n_f - 1} of the share workload ({sub.size} points, every line, "
                      f"cal-L={L}), forward filter, {dt:.1f} s"}


def host_cpu():
    """Model name and logical CPU count of the host, from /proc/cpuinfo."""
    try:
        with open("/proc/cpuinfo") as fh:
            names = [l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")]
        return f"{names[0]} ({len(names)} logical CPUs visible)" if names else None
    except OSError:
        return None


def calibrate_copy(torch, x, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_bytes_each": 2 * x.numel() * 8, "reps": reps}


def bench_patches(torch, steps, stream, n_theta_choices=(16, 32, 64, 128), force=None):
    """64 uneven patches: one tuned graph-replayed batch launch against one plan
    (two kernel launches) per patch, forward in place, same buffers.
    n_theta_choices: the patches' n_theta (n_phi = 2 n_theta).  force: a
    schedule (split, workgroups per CU, theta tiles, phi groups) set instead of
    the tuner's; then only the batched forward is timed."""
    import tempfile
    from paper_2305_01537_amd import synth
    from paper_2305_01537_amd.filter import Batch, Plan
    pts = synth.patches(with_values=False, n_theta_choices=n_theta_choices)
    g = torch.Generator(device="cuda").manual_seed(4)
    xs = [torch.randn((p.n_fields, p.n_r, p.n_theta, p.n_phi), dtype=torch.float64, device="cuda",
                      generator=g) for p in pts]
    if force is not None:
        batch = Batch(pts)
        batch.set_schedule_ex(split=force[0], workgroups_per_cu=force[1], fused=True,
                              theta_tiles=force[2], phi_groups=force[3])
        st = batch.stats()
        ms_b = time_loop(torch, lambda b: batch.apply(b, outs=b), [xs], steps, 3, stream)
        assert batch.status() == 0
        out = {"patches": len(pts), "algorithmic_bytes": st["bytes_fused_inplace"],
               "batched_forward_ms": ms_b,
               "batched_GBps": st["bytes_fused_inplace"] / (ms_b * 1e-3) / 1e9,
               "schedule": batch.get_schedule()}
        batch.close()
        return out
    with tempfile.TemporaryDirectory() as d:
        batch = Batch(pts, tune_cache=os.path.join(d, "tune.json"))
    sched = batch.get_schedule()
    st = batch.stats()
    ms_b = time_loop(torch, lambda b: batch.apply(b, outs=b), [xs], steps, 3, stream)
    ms_ba = time_loop(torch, lambda b: batch.apply(b, outs=b, adjoint=True), [xs], steps, 3, stream)
    # the tuner's choice of fused items, and the same schedule with the other choice
    tuned_fused = batch.get_fused()[0]
    batch.set_fused(not tuned_fused)
    st_alt = batch.stats()
    ms_alt = time_loop(torch, lambda b: batch.apply(b, outs=b), [xs], steps, 3, stream)
    batch.set_fused(tuned_fused)
    plans = [Plan(p.n_r, p.n_theta, p.n_phi, p.n_fields, parity=p.parity, L=p.L, rho=p.rho)
             for p in pts]

    def per_patch(b):
        for pl, x in zip(plans, b):
            pl.apply(x, out=x)
    ms_pp = time_loop(torch, per_patch, [xs], steps, 3, stream)
    assert batch.status() == 0
    out = {
        "patches": len(pts), "points": st["n_points"],
        "algorithmic_bytes": st["bytes_fused_inplace"],
        "batched_forward_ms": ms_b, "batched_adjoint_ms": ms_ba, "per_patch_launch_ms": ms_pp,
        "tuned_fused_items": tuned_fused, "shells_fused": st["shells_fused"],
        "other_setting": {"fused_items": not tuned_fused, "forward_ms": ms_alt,
                          "shells_fused": st_alt["shells_fused"],
                          "algorithmic_bytes": st_alt["bytes_fused_inplace"]},
        "batched_points_per_s": st["n_points"] / (ms_b * 1e-3),
        "batched_GBps": st["bytes_fused_inplace"] / (ms_b * 1e-3) / 1e9,
        "batched_over_per_patch_speedup": ms_pp / ms_b,
        "schedule": sched,
    }
    for pl in plans:
        pl.close()
    batch.close()
    return out


def bench_grmhd(torch, steps, stream):
    """The grmhd grid (24 x 128 x 64 x 128, 201 MB, paper cutoff): shells fit in
    LDS, so the plan fuses the theta-filtered shells; timed fused and as two
    passes, forward and adjoint in place.  Five rotated buffers (1 GB) keep the
    data out of the 256 MB last-level cache."""
    from paper_2305_01537_amd import synth
    from paper_2305_01537_amd.filter import Plan
    w = synth.workload("grmhd")
    F, R, T, P = w.shape
    plan = Plan(R, T, P, F, parity=w.parity, L=w.L, rho=w.rho)
    st = plan.stats()
    x0 = torch.from_numpy(w.x).cuda()
    bufs = [x0] + [x0.clone() for _ in range(4)]
    out = {"workload": f"grmhd: {F} x {R} x {T} x {P}, cal-L={float(w.L[0])}",
           "points": st["n_points"], "shells_fused": st["shells_fused"],
           "bytes_two_pass": st["bytes_forward_inplace"], "bytes_fused": st["bytes_fused_inplace"]}
    for fused in (True, False):
        plan.set_fused(fused)
        tag = "fused" if fused else "two_pass"
        ms_f = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 3, stream)
        ms_a = time_loop(torch, lambda b: plan.apply_adjoint(b, out=b), bufs, steps, 3, stream)
        nbytes = st["bytes_fused_inplace"] if fused else st["bytes_forward_inplace"]
        out[tag] = {"forward_ms": ms_f, "adjoint_ms": ms_a,
                    "points_per_s": st["n_points"] / (ms_f * 1e-3),
                    "GBps": nbytes / (ms_f * 1e-3) / 1e9}
    out["fused_speedup"] = out["two_pass"]["forward_ms"] / out["fused"]["forward_ms"]
    plan.close()
    del bufs, x0
    return out


def bench_chain(torch, steps, stream):
    """Differentiation on the chain workload (24 x 128 x 64 x 128, cal-L = 3):
    y_{k+1} = tanh(F y_k), K = 8, loss sum (y_K - t)^2, forward and backward
    through the adjoint filter, with and without checkpointing.  Reported per
    step and per filter call (checkpointed: 8 forward, 8 recomputed forward
    and 8 adjoint calls; plain: 8 forward and 8 adjoint)."""
    from paper_2305_01537_amd import synth
    from paper_2305_01537_amd.autograd import filter_chain
    from paper_2305_01537_amd.filter import Plan
    w = synth.workload("chain")
    F, R, T, P = w.shape
    plan = Plan(R, T, P, F, parity=w.parity, L=w.L, rho=w.rho)
    x = torch.from_numpy(w.x).cuda()
    t = torch.from_numpy(w.target).cuda()
    out = {"workload": f"chain: {F} x {R} x {T} x {P}, K = 8, tanh between filters"}
    for ck in (True, False):
        def step(_):
            xv = x.detach().requires_grad_(True)
            y = filter_chain(xv, plan, 8, checkpoint=ck)
            ((y - t) ** 2).sum().backward()
        ms = time_loop(torch, step, [None], steps, 2, stream)
        calls = 24 if ck else 16
        out["checkpointed" if ck else "plain"] = {"step_ms": ms, "filter_calls": calls,
                                                  "ms_per_filter_call_upper_bound": ms / calls}
    plan.close()
    return out


def bench_hybrid(torch, w, bufs, steps, stream):
    """The share with the paper's split of fields: 8 matter fields with the
    hybrid exponential/Gaussian switch at cal-L = 12, 16 metric fields
    exponential at cal-L = 3; forward in place, and with the decisions
    recorded (apply_ex) as the autograd forward does."""
    import numpy as np
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = w.shape
    kind = np.zeros(F, dtype=np.int32)
    kind[:8] = 3
    L = np.where(kind == 3, 12.0, 3.0)
    plan = Plan(R, T, P, F, parity=w.parity, L=L, rho=w.rho, kind=kind)
    st = plan.stats()
    ms_default = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 3, stream)
    # the plan's autotuner, as for the headline plan
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        tune = plan.tune(os.path.join(d, "tune.json"))
    schedule = {"theta_cols": plan.get_schedule()[0], "phi_lines": plan.get_schedule()[1],
                "overlap": plan.get_overlap(), **tune}
    ms = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 3, stream)
    ms_theta = time_loop(torch, lambda b: plan.apply_theta(b, out=b), bufs, steps, 2, stream)
    ms_phi = time_loop(torch, lambda b: plan.apply_phi(b, out=b), bufs, steps, 2, stream)
    th, ph = plan.decision_buffers()
    ms_rec = time_loop(torch, lambda b: plan.apply_ex(b, out=b, theta_dec=th, phi_dec=ph), bufs,
                       steps, 3, stream)
    # the recorded decisions replayed (no detector), as the adjoint of the
    # autograd backward runs them
    plan.apply_ex(bufs[0], out=bufs[1], theta_dec=th, phi_dec=ph)
    ms_rep = time_loop(torch, lambda b: plan.apply_ex(b, out=b, theta_dec=th, phi_dec=ph, replay=True),
                       bufs, steps, 3, stream)
    plan.close()
    return {"workload": "share, fields 0..7 hybrid (cal-L 12), 8..23 exponential (cal-L 3)",
            "forward_ms": ms, "forward_recording_ms": ms_rec, "forward_replay_ms": ms_rep,
            "forward_default_schedule_ms": ms_default,
            "theta_pass_ms": ms_theta, "phi_pass_ms": ms_phi, "schedule": schedule,
            "points_per_s": st["n_points"] / (ms * 1e-3),
            "GBps": st["bytes_forward_inplace"] / (ms * 1e-3) / 1e9,
            "algorithmic_bytes": st["bytes_forward_inplace"]}


def bench_mixed_radix(torch, steps, stream):
    """Lines with a radix-3 or radix-5 stage, on the angular grids of the
    paper's FFT(96) black-hole run (n_theta = 96, n_phi = 192: lines of 192,
    cal-L = 2) and of its explosion test (n_theta = 80, n_phi = 160: lines of
    160, cal-L = 4); 24 fields, rho = i + 1/2; at the paper's cutoff and dense
    (every line filtered, rho = 1, cal-L = 0.2): each pass and the forward
    filter in place."""
    import numpy as np
    from paper_2305_01537_amd.filter import Plan
    out = {}
    for grid, (F, R, T, P), L_paper in (("fft96_bh", (24, 128, 96, 192), 2.0),
                                        ("explosion", (24, 160, 80, 160), 4.0)):
        g = torch.Generator(device="cuda").manual_seed(P)
        x0 = torch.randn((F, R, T, P), dtype=torch.float64, device="cuda", generator=g)
        bufs = [x0, x0.clone()]
        parity = np.where(np.arange(F) % 3 == 2, -1, 1)
        res = {"shape": [F, R, T, P]}
        for name, L, rho in (("paper_cutoff", L_paper, None), ("dense", 0.2, np.ones(R))):
            plan = Plan(R, T, P, F, parity=parity, L=L, rho=rho)
            st = plan.stats()
            ms_t = time_loop(torch, lambda b: plan.apply_theta(b, out=b), bufs, steps, 5, stream)
            ms_p = time_loop(torch, lambda b: plan.apply_phi(b, out=b), bufs, steps, 5, stream)
            ms_f = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 5, stream)
            tb = 16 * st["theta_shells_active"] * T * P
            pb = 16 * st["phi_rings_active"] * P
            res[name] = {"cal_L": L, "forward_ms": ms_f,
                         "points_per_s": st["n_points"] / (ms_f * 1e-3),
                         "step_GBps": st["bytes_forward_inplace"] / (ms_f * 1e-3) / 1e9,
                         "theta_GBps": tb / (ms_t * 1e-3) / 1e9 if tb else None,
                         "phi_GBps": pb / (ms_p * 1e-3) / 1e9 if pb else None,
                         "active_theta_shells": st["theta_shells_active"],
                         "active_phi_rings": st["phi_rings_active"]}
            plan.close()
        out[grid] = res
        del bufs, x0
        torch.cuda.empty_cache()
    return out


def bench_short_lines(torch, steps, stream):
    """Dense cutoff (every line filtered) on grids with short lines,
    n_phi = 2 n_theta = 32, 64, 128, 24 fields and about 800 MB per buffer
    (two rotated buffers): the throughput of each pass and of the fused
    shells.  These are the sizes where a dense circulant on the matrix cores
    would be cheapest; it moves the same bytes."""
    import numpy as np
    from paper_2305_01537_amd.filter import Plan
    out = {}
    F = 24
    for N in (32, 64, 128):
        T, P = N // 2, N
        R = int(800e6 // (F * T * P * 8))
        g = torch.Generator(device="cuda").manual_seed(N)
        x0 = torch.randn((F, R, T, P), dtype=torch.float64, device="cuda", generator=g)
        bufs = [x0, x0.clone()]
        # rho = 1 on every shell: cutoffs at the floor, every line filtered
        plan = Plan(R, T, P, F, parity=np.where(np.arange(F) % 3 == 2, -1, 1), L=0.2,
                    rho=np.ones(R))
        st = plan.stats()
        pts = F * R * T * P
        assert st["theta_shells_active"] == F * R and st["phi_rings_active"] == F * R * T
        ms_t = time_loop(torch, lambda b: plan.apply_theta(b, out=b), bufs, steps, 2, stream)
        ms_p = time_loop(torch, lambda b: plan.apply_phi(b, out=b), bufs, steps, 2, stream)
        ms_f = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 2, stream)
        plan.set_fused(False)
        ms_2 = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 2, stream)
        out[f"N{N}"] = {"shape": [F, R, T, P], "theta_GBps": 16 * pts / (ms_t * 1e-3) / 1e9,
                        "phi_GBps": 16 * pts / (ms_p * 1e-3) / 1e9,
                        "fused_forward_ms": ms_f, "fused_GBps": 16 * pts / (ms_f * 1e-3) / 1e9,
                        "two_pass_forward_ms": ms_2,
                        "fused_points_per_s": pts / (ms_f * 1e-3)}
        if N in (32, 64):
            # the theta pass as the circulant product on the matrix cores:
            # alone (two-pass path) and inside the fused shell kernel
            from paper_2305_01537_amd.filter import THETA_MFMA
            plan.set_theta_variant(THETA_MFMA)
            ms_mt = time_loop(torch, lambda b: plan.apply_theta(b, out=b), bufs, steps, 2, stream)
            ms_m2 = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 2, stream)
            plan.set_fused(True)
            ms_mf = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, steps, 2, stream)
            out[f"N{N}"]["mfma"] = {
                "theta_GBps": 16 * pts / (ms_mt * 1e-3) / 1e9, "theta_ms": ms_mt,
                "two_pass_forward_ms": ms_m2, "fused_forward_ms": ms_mf,
                "fused_GBps": 16 * pts / (ms_mf * 1e-3) / 1e9,
                "fft_theta_ms": ms_t}
        plan.close()
        del bufs, x0
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the filter never couples shells, so a multi-GPU run is a "
                                   "(field, r) split with no communication)"}))
        return 2
    import numpy as np
    import torch
    from paper_2305_01537_amd import synth
    from paper_2305_01537_amd.filter import Plan

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t_start = time.perf_counter()
    if args.patches_only:
        force = None
        if args.batch_schedule:
            force = tuple(int(v) for v in args.batch_schedule.split(","))
            assert len(force) == 4, "--batch-schedule takes four integers"
        print(json.dumps({"patches": bench_patches(torch, args.steps, stream, force=force)}), flush=True)
        return 0
    if args.grmhd_only:
        print(json.dumps({"grmhd": bench_grmhd(torch, args.steps, stream)}), flush=True)
        return 0
    if args.short_lines_only:
        print(json.dumps({"short_lines": bench_short_lines(torch, args.steps, stream)}), flush=True)
        return 0
    if args.mixed_radix_only:
        print(json.dumps({"mixed_radix": bench_mixed_radix(torch, args.steps, stream)}), flush=True)
        return 0

    log("generating the share workload (24 x 256 x 128 x 256, FP64)")
    w = synth.workload("share", L=args.L)
    if args.hybrid_only:
        x0 = torch.from_numpy(w.x).to(dev)
        bufs = [x0] + [x0.clone() for _ in range(3)]
        print(json.dumps({"hybrid": bench_hybrid(torch, w, bufs, args.steps, stream)}), flush=True)
        return 0
    F, R, T, P = w.shape
    plan = Plan(R, T, P, F, parity=w.parity, L=w.L, rho=w.rho)
    st = plan.stats()
    # the plan's autotuner picks its launch settings (before the workload is
    # uploaded: it times candidates on scratch fields of the plan's size)
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        tune = plan.tune(os.path.join(d, "tune.json"))
    plan_schedule = {"theta_cols": plan.get_schedule()[0], "phi_lines": plan.get_schedule()[1],
                     "overlap": plan.get_overlap(), **tune}
    log(f"plan tuner: {plan_schedule}")
    x0 = torch.from_numpy(w.x).to(dev)
    bufs = [x0] + [x0.clone() for _ in range(3)]
    torch.cuda.synchronize()
    log(f"workload ready in {time.perf_counter() - t_start:.1f} s; stats {st}")

    # ---- the timed region: K forward filters, in place -------------------
    warm_info = {}
    ms_fwd = time_loop(torch, lambda b: plan.apply(b, out=b), bufs, args.steps, args.warmup, stream,
                       info=warm_info)
    log(f"forward {ms_fwd:.4f} ms/step")
    points = st["n_points"]
    value = points / (ms_fwd * 1e-3)

    # ---- per-kernel launches (same data, same stream) for the roofline -----
    # each pass alone with the default launch shape (16-line theta sub-tiles,
    # 4 ring pairs per phi workgroup at these line lengths: the launches the
    # default step makes), whatever the tuner picked for the step, so that the
    # roofline kernel's launch is the same in every run and in the profiler
    # runs
    kplan = Plan(R, T, P, F, parity=w.parity, L=w.L, rho=w.rho)
    ms_theta = time_loop(torch, lambda b: kplan.apply_theta(b, out=b), bufs, args.steps, 2, stream)
    ms_phi = time_loop(torch, lambda b: kplan.apply_phi(b, out=b), bufs, args.steps, 2, stream)
    kplan.close()
    th_bytes = 16 * st["theta_shells_active"] * T * P
    ph_bytes = 16 * st["phi_rings_active"] * P
    if ms_phi >= ms_theta:
        dom, dom_ms, dom_bytes, units = "phi_kernel", ms_phi, ph_bytes, st["phi_rings_active"]
        unit_desc = f"{units} active rings x 256 points x 16 B"
    else:
        dom, dom_ms, dom_bytes, units = "theta_kernel", ms_theta, th_bytes, st["theta_shells_active"]
        unit_desc = f"{units} active shells x 128 x 256 points x 16 B"
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    step_gbps = st["bytes_forward_inplace"] / (ms_fwd * 1e-3) / 1e9
    log(f"theta {ms_theta:.4f} ms ({th_bytes / ms_theta / 1e6:.1f} GB/s), "
        f"phi {ms_phi:.4f} ms ({ph_bytes / ms_phi / 1e6:.1f} GB/s)")

    extra = {
        "plan_schedule": plan_schedule,
        "theta_pass_ms": ms_theta, "phi_pass_ms": ms_phi,
        "algorithmic_bytes_per_step": st["bytes_forward_inplace"],
        "step_GBps": step_gbps,
        "active_theta_shells": st["theta_shells_active"], "active_phi_rings": st["phi_rings_active"],
    }
    if not args.no_extra:
        ms_adj = time_loop(torch, lambda b: plan.apply_adjoint(b, out=b), bufs, args.steps, 2, stream)
        extra["adjoint_ms"] = ms_adj
        extra["adjoint_over_forward"] = ms_adj / ms_fwd
        log(f"adjoint {ms_adj:.4f} ms")
        # the same forward with the passes overlapped on a second stream (the
        # rings of theta-idle shells alongside the theta pass), with the
        # plan's phi launch shape and with full 256-lane phi workgroups
        mode = plan.get_overlap()
        tc, pl = plan.get_schedule()
        plan.set_overlap(1)
        extra["forward_overlapped_ms"] = time_loop(torch, lambda b: plan.apply(b, out=b), bufs,
                                                   args.steps, 2, stream)
        plan.set_schedule(phi_lines=16)
        extra["forward_overlapped_phi16_ms"] = time_loop(torch, lambda b: plan.apply(b, out=b), bufs,
                                                         args.steps, 2, stream)
        plan.set_schedule(theta_cols=tc, phi_lines=pl)
        plan.set_overlap(mode)
        extra["forward_again_ms"] = time_loop(torch, lambda b: plan.apply(b, out=b), bufs,
                                              args.steps, 2, stream)
        log(f"forward overlapped {extra['forward_overlapped_ms']:.4f} ms "
            f"({extra['forward_overlapped_phi16_ms']:.4f} ms with 16 ring pairs per phi workgroup), "
            f"again as tuned {extra['forward_again_ms']:.4f} ms")
        # plain per-field launches: one plan per field, its two passes on the
        # caller's stream
        plans = [Plan(R, T, P, 1, parity=w.parity[f:f + 1], L=w.L[f:f + 1], rho=w.rho) for f in range(F)]
        for p_ in plans:
            p_.set_overlap(0)

        def per_field(b):
            for f in range(F):
                v = b[f:f + 1]
                plans[f].apply(v, out=v)
        ms_pf = time_loop(torch, per_field, bufs, max(5, args.steps // 4), 2, stream)
        extra["per_field_launch_ms"] = ms_pf
        extra["batched_over_per_field_speedup"] = ms_pf / ms_fwd
        for p_ in plans:
            p_.close()
        # dense variant: every line of both passes active (cal-L = 0.2)
        dplan = Plan(R, T, P, F, parity=w.parity, L=0.2, rho=w.rho)
        dst = dplan.stats()
        ms_d = time_loop(torch, lambda b: dplan.apply(b, out=b), bufs, max(5, args.steps // 2), 2, stream)
        ms_dt = time_loop(torch, lambda b: dplan.apply_theta(b, out=b), bufs, max(5, args.steps // 2), 2, stream)
        ms_dp = time_loop(torch, lambda b: dplan.apply_phi(b, out=b), bufs, max(5, args.steps // 2), 2, stream)
        extra["dense"] = {
            "cal_L": 0.2, "forward_ms": ms_d,
            "points_per_s": points / (ms_d * 1e-3),
            "GBps": dst["bytes_forward_inplace"] / (ms_d * 1e-3) / 1e9,
            "theta_GBps": 16 * points / (ms_dt * 1e-3) / 1e9,
            "phi_GBps": 16 * points / (ms_dp * 1e-3) / 1e9,
        }
        log(f"dense: {extra['dense']}")
        dplan.close()
        log("timing the grmhd grid (fused shells)")
        extra["grmhd"] = bench_grmhd(torch, max(10, args.steps // 2), stream)
        log(f"grmhd: {extra['grmhd']}")
        log("timing the differentiation chain")
        extra["chain"] = bench_chain(torch, max(5, args.steps // 20), stream)
        log(f"chain: {extra['chain']}")
        log("timing the 64-patch batch")
        extra["patches"] = bench_patches(torch, max(10, args.steps // 2), stream)
        log(f"patches: {extra['patches']}")
        log("timing the hybrid filter on the share")
        extra["hybrid"] = bench_hybrid(torch, w, bufs, max(10, args.steps // 4), stream)
        log(f"hybrid: {extra['hybrid']}")
        # streaming reference: torch's own in-place elementwise kernel on the same buffers
        ms_ref = time_loop(torch, lambda b: b.mul_(1.0), bufs, max(5, args.steps // 2), 2, stream)
        extra["stream_reference_GBps"] = 16 * points / (ms_ref * 1e-3) / 1e9
    if args.calibrate:
        extra["calibration"] = calibrate_copy(torch, x0)
    del bufs, x0
    torch.cuda.empty_cache()
    if not args.no_extra:
        log("timing dense short-line grids")
        extra["short_lines"] = bench_short_lines(torch, max(10, args.steps // 2), stream)
        log(f"short lines: {extra['short_lines']}")
        log("timing radix-3 and radix-5 lines (96 x 192, 80 x 160)")
        extra["mixed_radix"] = bench_mixed_radix(torch, max(10, args.steps // 2), stream)
        log(f"mixed-radix lines: {extra['mixed_radix']}")
        for key, choices in (("patches_radix3", (24, 48, 96)), ("patches_radix5", (40, 80))):
            log(f"timing 64 patches with n_theta in {choices}")
            r = bench_patches(torch, max(10, args.steps // 2), stream, choices)
            extra[key] = {k: r[k] for k in ("points", "algorithmic_bytes", "batched_forward_ms",
                                            "per_patch_launch_ms", "batched_GBps",
                                            "batched_over_per_patch_speedup", "schedule")}
            extra[key]["n_theta_choices"] = list(choices)
            log(f"{key}: {extra[key]}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(w, args.L, args.cpu_seconds)
        log(f"cpu baseline {cpu}")
        extra["cpu_fft_baseline"] = cpu_fft_baseline(w, args.L, args.cpu_seconds / 2)
        log(f"cpu fft baseline {extra['cpu_fft_baseline']}")

    line = {
        "metric": "filtered field-points/s (FP64) & % HBM peak, batched vs per-field; adjoint/fwd",
        "value": value,
        "unit": "field-points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "clock_warmup_ms": warm_info["clock_warmup_ms"],
        "ms_per_step": ms_fwd,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"share: 24 fields x 256 r x 128 theta x 256 phi, FP64, "
                               f"paper cutoff cal-L={args.L} on rho=i+1/2, forward filter in place",
                   "fields": F, "n_r": R, "n_theta": T, "n_phi": P, "cal_L": args.L},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(dom, args.L),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": dom, "kernel_ms": dom_ms, "algorithmic_bytes": dom_bytes,
                     "units": unit_desc,
                     # the whole step (both passes, overlapped) at ms_per_step
                     "step_achieved": step_gbps, "step_frac": step_gbps / HBM_PEAK_GBS,
                     "step_algorithmic_bytes": st["bytes_forward_inplace"]},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    plan.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
