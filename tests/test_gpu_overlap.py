"""Overlapped passes on the GPU.

In place, and where shells are not fused, a plan runs the rings of shells the
theta pass leaves alone on a second stream, alongside the theta pass and the
rings of the theta-filtered shells on the caller's stream.  Each ring goes
through the same kernel either way, so the results must be bitwise those of
the plain two-pass path, and the fork/join must keep the call stream-ordered:
back-to-back calls on the same buffer, and a captured HIP graph replayed
several times, must see each other's results.
"""
import numpy as np
import pytest

import oracle
from paper_2305_01537_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-12
EXP, GAUSS, SHARP, HYBRID = 0, 1, 2, 3


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def fields(shape, seed):
    F, R, T, P = shape
    rng = np.random.default_rng(seed)
    theta, phi = synth.theta_grid(T), synth.phi_grid(P)
    x = np.empty(shape)
    for f in range(F):
        for i in range(R):
            x[f, i] = synth.angular_sum(rng, 10, theta, phi, lambda l: 1.0 / (l + 1))
    x += 1e-3 * rng.standard_normal(shape)
    parity = np.where(rng.random(F) < 0.5, 1, -1).astype(np.int32)
    x[parity < 0] *= np.sin(theta)[None, :, None]
    return x, parity


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    # n_phi = 2 n_theta = 256: shells too large to fuse
    ((3, 6, 128, 256), [EXP, GAUSS, SHARP], [21.0, 9.0, 15.0]),
    # n_phi != 2 n_theta: theta-filtered shells may keep identity rings
    ((3, 8, 32, 128), [EXP, SHARP, HYBRID], [3.0, 2.2, 1.5]),
]


@pytest.mark.parametrize("shape,kind,L", CASES)
def test_overlap_is_bitwise_the_two_pass_filter(torch_gpu, shape, kind, L):
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = shape
    x, parity = fields(shape, 111 + T)
    kind = np.array(kind, dtype=np.int32)
    L = np.array(L)
    plan = Plan(R, T, P, F, parity=parity, L=L, kind=kind)
    st = plan.stats()
    print(f"[gpu] overlap {shape}: theta shells {st['theta_shells_active']} of {F * R}", flush=True)
    assert 0 < st["theta_shells_active"] < F * R and plan.get_fused()[1] == 0
    assert plan.get_overlap() == 0
    for name, ref_fn in (("apply", oracle.forward), ("apply_adjoint", oracle.adjoint)):
        res = {}
        for ov in (2, 0):
            plan.set_overlap(ov)
            xd = torch.from_numpy(x).cuda()
            getattr(plan, name)(xd, out=xd)
            torch.cuda.synchronize()
            res[ov] = xd.cpu().numpy()
        assert np.array_equal(res[2], res[0]), name
        assert rel(res[2], ref_fn(x, parity=parity, L=L, kind=kind)) <= TOL, name
    plan.close()


def test_overlap_calls_stay_stream_ordered(torch_gpu):
    """Ten in-place calls back to back (each reads what the previous wrote,
    across both streams) equal ten calls with a synchronisation after each."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    shape = (2, 10, 128, 256)
    x, parity = fields(shape, 131)
    plan = Plan(10, 128, 256, 2, parity=parity, L=np.array([9.0, 12.0]))
    plan.set_overlap(2)
    a = torch.from_numpy(x).cuda()
    for _ in range(10):
        plan.apply(a, out=a)
    torch.cuda.synchronize()
    b = torch.from_numpy(x).cuda()
    plan.set_overlap(0)
    for _ in range(10):
        plan.apply(b, out=b)
        torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_overlap_in_a_captured_graph(torch_gpu):
    """The fork and join are captured with the call: every replay of the graph
    (with eager work and synchronisation between replays) equals the eager
    call on the same input."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    shape = (2, 10, 128, 256)
    x, parity = fields(shape, 141)
    plan = Plan(10, 128, 256, 2, parity=parity, L=np.array([9.0, 12.0]))
    plan.set_overlap(2)
    eager = torch.from_numpy(x).cuda()
    plan.apply(eager, out=eager)
    torch.cuda.synchronize()
    buf = torch.from_numpy(x).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.apply(buf, out=buf)                 # warm-up call before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.apply(buf, out=buf)
    src = torch.from_numpy(x).cuda()
    for k in range(4):
        buf.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(buf, eager), k
        _ = (src * 2.0).sum().item()              # eager work between replays
    plan.close()


def test_set_overlap_modes(torch_gpu):
    from paper_2305_01537_amd import _lib
    from paper_2305_01537_amd.filter import Plan
    plan = Plan(2, 16, 32, 1, parity=[1], L=[0.5])
    lib = _lib.load()
    assert lib.sphfilt_plan_set_overlap(plan._h, 3) == _lib.EINVAL
    assert lib.sphfilt_plan_set_overlap(plan._h, -1) == _lib.EINVAL
    assert lib.sphfilt_plan_get_overlap(plan._h, None) == _lib.EINVAL
    for m in (0, 1, 2):
        plan.set_overlap(m)
        assert plan.get_overlap() == m
    plan.close()


def test_overlap_records_and_replays_hybrid_decisions(torch_gpu):
    """With the other fields' idle-shell rings on the second stream, the hybrid
    field's decisions (a hybrid shell is never idle) and the replayed adjoint
    are bitwise those of the one-stream call."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    shape, kind, L = CASES[1]
    F, R, T, P = shape
    x, parity = fields(shape, 151)
    x[2, 6, 3, :] = np.where(np.arange(P) < 40, 0.0, 1.5)      # a ring jump in the hybrid field
    plan = Plan(R, T, P, F, parity=parity, L=np.array(L), kind=np.array(kind, dtype=np.int32))
    g = np.random.default_rng(152).standard_normal(shape)
    res = {}
    for ov in (2, 0):
        plan.set_overlap(ov)
        th, ph = plan.decision_buffers()
        y = torch.from_numpy(x).cuda()
        plan.apply_ex(y, out=y, theta_dec=th, phi_dec=ph)
        z = torch.from_numpy(g).cuda()
        plan.apply_ex(z, out=z, adjoint=True, theta_dec=th, phi_dec=ph, replay=True)
        torch.cuda.synchronize()
        res[ov] = [t.cpu().numpy() for t in (y, th, ph, z)]
    for a, b in zip(res[2], res[0]):
        assert np.array_equal(a, b)
    assert res[2][2][2].any()
    plan.close()


@pytest.mark.parametrize("shape,overlap", [((2, 10, 128, 256), 2), ((2, 10, 128, 256), 0),
                                           ((3, 6, 64, 128), 0)])
def test_one_plan_on_two_streams(torch_gpu, shape, overlap):
    """A plan keeps no scratch, so one plan may run on several streams at once:
    forward and adjoint calls on two streams without synchronisation (in place,
    each stream on its own fields; overlapped passes, plain passes, fused
    shells) give bitwise what the same calls give one after another."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    F, R, T, P = shape
    xa, parity = fields(shape, 171)
    xb, _ = fields(shape, 172)
    plan = Plan(R, T, P, F, parity=parity, L=np.full(F, 9.0))
    plan.set_overlap(overlap)
    print(f"[gpu] one plan, two streams {shape} overlap {overlap}", flush=True)

    def call(d):
        plan.apply(d, out=d)
        plan.apply_adjoint(d, out=d)

    ref = []
    for x in (xa, xb):
        d = torch.from_numpy(x).cuda()
        for _ in range(5):
            call(d)
        torch.cuda.synchronize()
        ref.append(d.cpu().numpy())
    bufs = [torch.from_numpy(x).cuda() for x in (xa, xb)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for _ in range(5):                             # the two streams' calls interleave
        for s, d in zip(streams, bufs):
            with torch.cuda.stream(s):
                call(d)
    torch.cuda.synchronize()
    for d, r in zip(bufs, ref):
        assert np.array_equal(d.cpu().numpy(), r)
    plan.close()


def test_one_plan_from_two_host_threads(torch_gpu):
    """Two host threads call one plan at once (the binding releases the
    interpreter lock during the library call), each on its own stream and
    fields, forward and adjoint in place: every result equals the same calls
    made one after another."""
    import threading
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    shape = (2, 10, 128, 256)
    xs = [fields(shape, s)[0] for s in (181, 182)]
    _, parity = fields(shape, 181)
    plan = Plan(10, 128, 256, 2, parity=parity, L=np.full(2, 9.0))
    plan.set_overlap(2)

    def calls(d):
        for _ in range(10):
            plan.apply(d, out=d)
            plan.apply_adjoint(d, out=d)

    ref = []
    for x in xs:
        d = torch.from_numpy(x).cuda()
        calls(d)
        torch.cuda.synchronize()
        ref.append(d.cpu().numpy())
    bufs = [torch.from_numpy(x).cuda() for x in xs]
    torch.cuda.synchronize()
    errors = []

    def worker(d):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                calls(d)
            s.synchronize()
        except Exception as e:          # reported by the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(d,)) for d in bufs]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for d, r in zip(bufs, ref):
        assert np.array_equal(d.cpu().numpy(), r)
    plan.close()


def test_plans_in_a_captured_graph(torch_gpu):
    """Forward and adjoint calls of a fused-shell plan and of a two-pass plan
    captured in one graph: every replay (with eager work and synchronisation
    between replays) equals the same calls made eagerly."""
    torch = torch_gpu
    from paper_2305_01537_amd.filter import Plan
    xa, pa = fields((2, 6, 32, 64), 191)
    xb, pb = fields((2, 5, 64, 256), 192)
    fused = Plan(6, 32, 64, 2, parity=pa, L=np.array([2.0, 0.7]))
    assert fused.get_fused()[1] > 0
    plain = Plan(5, 64, 256, 2, parity=pb, L=np.array([2.0, 0.7]))

    def calls(a, b):
        fused.apply(a, out=a)
        plain.apply(b, out=b)
        fused.apply_adjoint(a, out=a)
        plain.apply_adjoint(b, out=b)

    ea, eb = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    calls(ea, eb)
    torch.cuda.synchronize()
    a, b = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls(a, b)                                  # warm-up before the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls(a, b)
    sa, sb = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    for k in range(4):
        a.copy_(sa)
        b.copy_(sb)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(a, ea) and torch.equal(b, eb), k
        _ = (sa * 2.0).sum().item()                   # eager work between replays
    fused.close()
    plain.close()
