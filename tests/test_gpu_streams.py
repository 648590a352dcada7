"""Distinct plans are independent: plans working at the same time on streams
of their own, enqueued from one host thread or from several, give exactly
the results of the same calls made one after another; plans created from
several host threads at once equal plans created one by one."""
import threading

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GRIDS = {
    "c2": synth.config_desc("c2"),
    "ragged": synth.GridDesc(nt=301, nx=77, dt=0.004, x0=0.1, dx=0.025, ntau=250, nq=61,
                             tau0=0.05, dtau=0.0045, q0=0.22, dq=0.0075, oversample=2.0),
    "c1": synth.config_desc("c1"),
}
ROUNDS = 4


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def make_cases():
    from paper_1604_07651_amd.hrt import Plan
    cases = []
    for k, (name, desc) in enumerate(GRIDS.items()):
        plan = Plan(desc)
        f, g = synth.random_pair(desc, 60 + k)
        cases.append((name, plan, to_gpu(f), to_gpu(g)))
    return cases


def serial_results(cases):
    out = {}
    for name, plan, F, G in cases:
        gn, fn = plan.normal(F)
        out[name] = (plan.forward(F), plan.adjoint(G), gn, fn)
    torch.cuda.synchronize()
    return out


def run_on(plan, F, G, outs, rounds):
    g_out, f_out, gn_out, fn_out = outs
    for _ in range(rounds):
        plan.forward(F, out=g_out)
        plan.adjoint(G, out=f_out)
        plan.normal(F, g=gn_out, out=fn_out)


def check(ref, outs, name):
    for r, o, what in zip(ref, outs, ("forward", "adjoint", "normal g", "normal f")):
        assert torch.equal(o, r), f"{name}: {what} differs from the serial result"


def fresh_outputs(ref):
    return [torch.full_like(r, float("nan")) for r in ref]


def test_plans_on_concurrent_streams_one_thread():
    cases = make_cases()
    ref = serial_results(cases)
    streams = [torch.cuda.Stream() for _ in cases]
    outs = {name: fresh_outputs(ref[name]) for name, *_ in cases}
    torch.cuda.synchronize()
    print("[gpu] plans interleaved on streams", flush=True)
    # round-robin enqueue: every stream has work in flight beside the others
    for _ in range(ROUNDS):
        for (name, plan, F, G), s in zip(cases, streams):
            with torch.cuda.stream(s):
                run_on(plan, F, G, outs[name], 1)
    torch.cuda.synchronize()
    for name, *_ in cases:
        check(ref[name], outs[name], name)
    for _, plan, *_ in cases:
        plan.close()


def test_plans_on_concurrent_streams_many_threads():
    cases = make_cases()
    ref = serial_results(cases)
    outs = {name: fresh_outputs(ref[name]) for name, *_ in cases}
    torch.cuda.synchronize()
    errors = []

    def worker(name, plan, F, G):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                run_on(plan, F, G, outs[name], ROUNDS)
            s.synchronize()
        except Exception as e:  # reported in the main thread
            errors.append(f"{name}: {e!r}")

    print("[gpu] plans from host threads", flush=True)
    threads = [threading.Thread(target=worker, args=c) for c in cases]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a worker thread did not finish"
    torch.cuda.synchronize()
    assert not errors, errors
    for name, *_ in cases:
        check(ref[name], outs[name], name)
    for _, plan, *_ in cases:
        plan.close()


def test_plans_created_from_many_threads():
    from paper_1604_07651_amd.hrt import Plan
    desc = GRIDS["ragged"]
    f, _ = synth.random_pair(desc, 70)
    F = to_gpu(f)
    base = Plan(desc)
    ref = base.forward(F)
    torch.cuda.synchronize()
    plans, errors = [None] * 4, []

    def make(i):
        try:
            plans[i] = Plan(GRIDS["c1"] if i % 2 else desc)
        except Exception as e:
            errors.append(repr(e))

    print("[gpu] plan creation from host threads", flush=True)
    threads = [threading.Thread(target=make, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a plan creation did not finish"
    assert not errors, errors
    for i in (0, 2):
        got = plans[i].forward(F)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
    for p in plans + [base]:
        p.close()
