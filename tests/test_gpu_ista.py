"""GPU soft-thresholding iterations (Section 3, eqs. iters and itersmd)
through the C ABI against the float64 oracle; their HIP-graph capture
against eager launches; the float64 power iteration; and the autograd
backward of the forward transform checked by finite differences."""
import numpy as np
import pytest

import synth
from oracle import ista as oista
from oracle import logpolar

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

C1 = synth.config_desc("c1")
_cache = {}


def setup(name="c1"):
    if name not in _cache:
        from paper_1604_07651_amd.hrt import Plan
        desc = synth.config_desc(name)
        print(f"[plan] {name}", flush=True)
        _cache[name] = (desc, Plan(desc), logpolar.LogPolarOracle(desc) if name == "c1" else None)
    return _cache[name]


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def data_mask(desc, frac, seed):
    keep = synth.trace_mask(desc.nx, frac, seed)
    return np.repeat(keep[:, None], desc.nt, axis=1).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


@pytest.mark.parametrize("masked", [False, True])
def test_ista_iterations_match_oracle(masked):
    desc, plan, ora = setup()
    f = synth.config_gather("c1")
    mask = data_mask(desc, 0.5, 11) if masked else None
    if masked:
        f = f * mask
    lam = oista.power_norm2(ora.forward, ora.adjoint, plan.data_shape, iters=100, seed=2)
    c2 = 0.99 / lam
    mu = 0.05 * np.abs(ora.forward(f)).max()
    iters = 20
    ref = oista.ista(ora.forward, ora.adjoint, f, iters, c2, mu, mask)
    g = torch.zeros(plan.radon_shape, device="cuda")
    print(f"[gpu] ista c1 masked={masked}", flush=True)
    plan.ista_iterate(to_gpu(f), g, iters, c2, mu,
                      mask=to_gpu(mask) if masked else None)
    torch.cuda.synchronize()
    r = rel(g.cpu().numpy(), ref)
    print(f"  ista rel-L2 {r:.2e}", flush=True)
    assert r <= 2e-5


def test_opnorm2_matches_oracle():
    desc, plan, ora = setup()
    print("[gpu] opnorm2", flush=True)
    lam = plan.opnorm2(iters=200, seed=5)
    ref = oista.power_norm2(ora.forward, ora.adjoint, plan.data_shape, iters=200, seed=6)
    print(f"  ||R||^2 gpu {lam:.8e} oracle {ref:.8e}", flush=True)
    assert abs(lam - ref) <= 1e-4 * ref


def test_graph_replays_match_eager():
    desc, plan, ora = setup()
    f = to_gpu(synth.config_gather("c1"))
    mask = to_gpu(data_mask(desc, 0.5, 12))
    f = f * mask
    g0 = torch.from_numpy(synth.random_pair(desc, 13)[1].astype(np.float32)).cuda() * 0.01
    c2, mu, iters = 0.5 / plan.opnorm2(iters=20), 1e-3, 7
    g_eager = g0.clone()
    plan.ista_iterate(f, g_eager, iters, c2, mu, mask=mask)
    torch.cuda.synchronize()
    g_graph = torch.empty_like(g0)
    print("[gpu] ista graph capture", flush=True)
    gr = plan.ista_graph(f, g_graph, iters, c2, mu, mask=mask)
    for rep in range(3):
        g_graph.copy_(g0)
        torch.cuda.synchronize()
        gr.launch()
        torch.cuda.synchronize()
        print(f"  replay {rep}", flush=True)
        assert torch.equal(g_graph, g_eager)
        # unrelated eager work between replays
        plan.forward(f)
        torch.cuda.synchronize()
    gr.close()


def test_ista_argument_errors():
    desc, plan, ora = setup()
    f = torch.zeros(plan.data_shape, device="cuda")
    g = torch.zeros(plan.radon_shape, device="cuda")
    from paper_1604_07651_amd import _lib
    import ctypes as C
    lib = plan._lib
    wd = torch.zeros(plan.data_shape, device="cuda")
    # overlapping scratch and panel, negative step
    st = lib.hrt_ista_iterate(plan._h, C.c_void_p(f.data_ptr()), None, C.c_void_p(g.data_ptr()),
                              C.c_void_p(wd.data_ptr()), C.c_void_p(g.data_ptr()), 1,
                              C.c_float(0.1), C.c_float(0.0), None)
    assert st == 1
    st = lib.hrt_ista_iterate(plan._h, C.c_void_p(f.data_ptr()), None, C.c_void_p(g.data_ptr()),
                              C.c_void_p(wd.data_ptr()),
                              C.c_void_p(torch.zeros(plan.radon_shape, device="cuda").data_ptr()),
                              1, C.c_float(-0.1), C.c_float(0.0), None)
    assert st == 1


def test_autograd_backward_by_finite_differences_c3():
    """L(f) = <R f, w> at the full-size gather: autograd's gradient is the
    adjoint R^T w, and central differences along 64 seeded directions
    (seeds 300-363) agree with <grad, d>."""
    from paper_1604_07651_amd.hrt import HRTFunction
    desc, plan, _ = setup("c3")
    f0 = to_gpu(synth.config_gather("c3"))
    w = to_gpu(np.random.default_rng(299).standard_normal(plan.radon_shape))
    f = f0.clone().requires_grad_(True)
    print("[gpu] autograd c3", flush=True)
    L = (HRTFunction.apply(f, plan) * w).sum()
    L.backward()
    grad = f.grad.detach()
    assert torch.equal(grad, plan.adjoint(w))

    def loss(x):
        return torch.sum(plan.forward(x).double() * w.double()).item()

    errs = []
    for s in range(300, 364):
        d = to_gpu(np.random.default_rng(s).standard_normal(plan.data_shape))
        # L is linear, so any step is exact in exact arithmetic; a step the
        # size of f keeps float32 cancellation in L(f + eps d) - L(f - eps d) small
        eps = (f0.norm() / d.norm()).item()
        fd = (loss(f0 + eps * d) - loss(f0 - eps * d)) / (2 * eps)
        an = torch.sum(grad.double() * d.double()).item()
        errs.append(abs(fd - an) / abs(an))
    print(f"  FD max rel err over 64 directions {max(errs):.2e}", flush=True)
    assert max(errs) <= 1e-3


def test_demultiple_matches_oracle():
    from oracle import demultiple
    desc, plan, ora = setup()
    f, prim, mult = synth.demultiple_gather(desc, 21)
    g = synth.random_pair(desc, 22)[1] * 0.01
    for qb0, slope in ((1 / 2.05, 0.0), (0.4, 0.08)):
        print(f"[gpu] demultiple border {qb0:.4f} + {slope} tau", flush=True)
        out = plan.demultiple(to_gpu(f), to_gpu(g), qb0, slope)
        torch.cuda.synchronize()
        ref = demultiple.demultiple(ora.adjoint, desc, f, g, qb0, slope)
        r = rel(out.cpu().numpy(), ref)
        print(f"  demultiple rel-L2 {r:.2e}", flush=True)
        assert r <= 1e-5
        # the removed part alone (zero gather: the output is minus the
        # adjoint of the muted panel)
        zero = np.zeros_like(f)
        out0 = plan.demultiple(to_gpu(zero), to_gpu(g), qb0, slope)
        torch.cuda.synchronize()
        r = rel(out0.cpu().numpy(), demultiple.demultiple(ora.adjoint, desc, zero, g, qb0, slope))
        print(f"  removed part rel-L2 {r:.2e}", flush=True)
        assert r <= 1e-5


def test_demultiple_pipeline_attenuates_multiples_on_gpu():
    """ISTA (30 iterations, one HIP graph) then the Radon-domain mute and
    subtraction, all on the GPU: multiples attenuated as in the oracle."""
    from paper_1604_07651_amd.hrt import ista
    desc, plan, ora = setup()
    f, prim, mult = synth.demultiple_gather(desc, 21)
    F = to_gpu(f)
    mu = 0.01 * plan.forward(F).abs().max().item()
    print("[gpu] demultiple pipeline", flush=True)
    g = ista(plan, F, iters=30, mu=mu, graph=True)
    out = plan.demultiple(F, g, 1 / 2.05).cpu().numpy()
    before = np.linalg.norm(f - prim)
    after = np.linalg.norm(out - prim)
    print(f"  primaries error {after / before:.3f} of the input's", flush=True)
    assert after <= 0.6 * before
