"""Behaviour flags of hrt_desc and the allocation-failure hook, through the
C ABI:

* HRT_ACCUMULATE_OUTPUT: the forward, the adjoint, the allocation-free
  forward and the split transforms add into their output (out = y0 + R f,
  compared with y0 + the overwriting call's result, float32 addition); the
  plain plan's call with the flag equals the oracle plus y0; hrt_normal and
  batches refuse the flag;
* HRT_DETERMINISTIC: accepted; two runs give the same bits (as every run
  does);
* HRT_FAIL_ALLOC=k: the k-th device allocation of a plan creation fails with
  HRT_ERR_OOM for every k up to the plan's allocation count, nothing leaks,
  and a creation without the hook works afterwards."""
import os

import numpy as np
import pytest

import synth
from oracle import logpolar

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

ACC = 256
DET = 512


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("name", ["c1", "ragged"])
def test_accumulate_output_adds(name):
    from paper_1604_07651_amd.hrt import Plan
    desc = synth.config_desc("c1") if name == "c1" else synth.GridDesc(
        nt=301, nx=77, dt=0.004, x0=0.1, dx=0.025, ntau=250, nq=61, tau0=0.05,
        dtau=0.0045, q0=0.22, dq=0.0075)
    plain = Plan(desc)
    acc = Plan(desc, flags=ACC)
    f, g = synth.random_pair(desc, 51)
    y0, x0 = synth.random_pair(desc, 52)  # y0 is data-shaped, x0 Radon-shaped
    F, G = to_gpu(f), to_gpu(g)
    print(f"[gpu] accumulate {name}", flush=True)
    gf = plain.forward(F)
    fa = plain.adjoint(G)
    out_g = to_gpu(x0)
    acc.forward(F, out=out_g)
    out_f = to_gpu(y0)
    acc.adjoint(G, out=out_f)
    gn = torch.empty_like(gf)
    acc.forward_noalloc(F, out=gn.copy_(to_gpu(x0)))
    torch.cuda.synchronize()
    assert torch.equal(out_g, to_gpu(x0) + gf)
    assert torch.equal(out_f, to_gpu(y0) + fa)
    assert torch.equal(gn, to_gpu(x0) + gf)
    ora = logpolar.LogPolarOracle(desc)
    ref = ora.forward(f) + x0.astype(np.float32)
    r = np.linalg.norm(out_g.double().cpu().numpy() - ref) / np.linalg.norm(ref)
    assert r <= 1e-5
    from paper_1604_07651_amd import _lib
    with pytest.raises(_lib.HrtError):
        acc.normal(F)
    plain.close()
    acc.close()


def test_accumulate_output_split_and_batch_refusal():
    from paper_1604_07651_amd import _lib
    from paper_1604_07651_amd.hrt import Batch, Split, split_edges
    desc = synth.config_desc("c1")
    te, qe = split_edges(desc)
    s0 = Split(desc, te, qe)
    s1 = Split(desc, te, qe, flags=ACC)
    f, g = synth.random_pair(desc, 61)
    y0, x0 = synth.random_pair(desc, 62)
    F, G = to_gpu(f), to_gpu(g)
    print("[gpu] accumulate split", flush=True)
    gs = s0.forward(F)
    fs = s0.adjoint(G)
    out_g = to_gpu(x0)
    s1.forward(F, out=out_g)
    out_f = to_gpu(y0)
    s1.adjoint(G, out=out_f)
    torch.cuda.synchronize()
    # the parts add one after another onto x0: the same sums in another
    # order than x0 + (sum of parts), so float32 rounding may differ
    for got, want in ((out_g, to_gpu(x0) + gs), (out_f, to_gpu(y0) + fs)):
        err = (torch.linalg.norm((got - want).double()) / torch.linalg.norm(want.double())).item()
        assert err <= 1e-6
    s0.close()
    s1.close()
    with pytest.raises(_lib.HrtError):
        Batch([desc], flags=ACC)


def test_deterministic_flag_accepted_and_runs_repeat():
    from paper_1604_07651_amd.hrt import Plan
    desc = synth.config_desc("c2")
    p0 = Plan(desc)
    p1 = Plan(desc, flags=DET)
    f, g = synth.random_pair(desc, 71)
    F, G = to_gpu(f), to_gpu(g)
    print("[gpu] deterministic", flush=True)
    outs = [(p.forward(F), p.adjoint(G)) for p in (p0, p1, p0, p1)]
    torch.cuda.synchronize()
    for a, b in outs[1:]:
        assert torch.equal(a, outs[0][0]) and torch.equal(b, outs[0][1])
    p0.close()
    p1.close()


def test_injected_allocation_failures_clean_up(monkeypatch):
    from paper_1604_07651_amd import _lib
    from paper_1604_07651_amd.hrt import Plan
    desc = synth.config_desc("c1")
    torch.cuda.synchronize()
    Plan(desc).close()  # the runtime's own first-use allocations
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    print("[gpu] allocation failures", flush=True)
    k = 0
    while True:
        k += 1
        assert k < 200, "plan creation never completed"
        monkeypatch.setenv("HRT_FAIL_ALLOC", str(k))
        try:
            p = Plan(desc)
        except _lib.HrtError as e:
            assert e.status == 3, e  # HRT_ERR_OOM
            continue
        p.close()
        break
    print(f"  a plan makes {k - 1} device allocations; each failure cleaned up", flush=True)
    assert k > 10
    monkeypatch.delenv("HRT_FAIL_ALLOC")
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 <= 4 << 20, f"{(free0 - free1) / 2**20:.1f} MiB not returned"
    p = Plan(desc)
    f = to_gpu(synth.random_pair(desc, 3)[0])
    g = p.forward(f)
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    p.close()
