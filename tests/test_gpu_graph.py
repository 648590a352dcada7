"""HIP-graph capture of the plain transforms: hrt_forward, hrt_adjoint and
hrt_normal launch only on the caller's stream and never allocate or
synchronise, so a caller can capture them (here through torch's graph
capture, which runs the library calls on its capture stream).  Every replay,
with eager work and synchronisations between replays, must equal the eager
calls bit for bit."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_captured_transforms_replay_like_eager(name):
    from paper_1604_07651_amd.hrt import Plan
    desc = synth.config_desc(name)
    plan = Plan(desc)
    f, g = synth.random_pair(desc, 81)
    F = torch.from_numpy(f.astype(np.float32)).cuda()
    G = torch.from_numpy(g.astype(np.float32)).cuda()
    # eager reference
    g_ref = plan.forward(F)
    f_ref = plan.adjoint(G)
    gn_ref, fn_ref = plan.normal(F)
    torch.cuda.synchronize()
    # outputs the graph writes
    g_out = torch.empty_like(g_ref)
    f_out = torch.empty_like(f_ref)
    gn_out = torch.empty_like(gn_ref)
    fn_out = torch.empty_like(fn_ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on a side stream, as torch advises
        plan.forward(F, out=g_out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    print(f"[gpu] capture {name}", flush=True)
    with torch.cuda.graph(graph):
        plan.forward(F, out=g_out)
        plan.adjoint(G, out=f_out)
        plan.normal(F, g=gn_out, out=fn_out)
    for rep in range(3):
        for t in (g_out, f_out, gn_out, fn_out):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        print(f"[gpu] replay {rep}", flush=True)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g_out, g_ref)
        assert torch.equal(f_out, f_ref)
        assert torch.equal(gn_out, gn_ref)
        assert torch.equal(fn_out, fn_ref)
        plan.forward(G.new_zeros(plan.data_shape))  # eager work between replays
        torch.cuda.synchronize()
    del graph
    plan.close()
