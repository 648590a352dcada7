"""Uneven batches (one launch per kernel for all gathers) through the C ABI:
every gather's result equals the single-gather call bit for bit, and the
single-gather calls match the FP64 oracle (test_gpu_parity)."""
import numpy as np
import pytest

import synth
from oracle import logpolar

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DESCS = [
    synth.config_desc("c1"),
    synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                   tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5),
    synth.GridDesc(nt=301, nx=77, dt=0.004, x0=0.1, dx=0.025, ntau=250,
                   nq=61, tau0=0.05, dtau=0.0045, q0=0.22, dq=0.0075),
    synth.GridDesc(nt=16, nx=16, dt=0.01, x0=0.0, dx=0.02, ntau=16, nq=16,
                   tau0=0.0, dtau=0.01, q0=0.25, dq=(1 / 1.5 - 0.25) / 15),
    synth.config_desc("c2"),
    # a 4320-point log-radius axis: the column kernel's paths for columns it
    # cannot hold in registers or transform in place, in the batched launch
    synth.GridDesc(nt=6000, nx=96, dt=0.0007, x0=0.0, dx=1.5 / 95, ntau=6000, nq=96,
                   tau0=0.0, dtau=0.0007, q0=0.25, dq=(1 / 1.5 - 0.25) / 95),
]


def run_batch(descs, seed):
    from paper_1604_07651_amd.hrt import Batch, Plan
    print(f"[batch] {len(descs)} gathers", flush=True)
    b = Batch(descs)
    pairs = [synth.random_pair(d, seed + i, dtype=np.float32) for i, d in enumerate(descs)]
    F = b.pack_data([p[0] for p in pairs])
    G = b.pack_radon([p[1] for p in pairs])
    gb = b.forward(F)
    fb = b.adjoint(G)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        plan = Plan(d)
        g1 = plan.forward(b.unpack_data(F)[i].contiguous())
        f1 = plan.adjoint(b.unpack_radon(G)[i].contiguous())
        torch.cuda.synchronize()
        print(f"  gather {i} {d.nt}x{d.nx}", flush=True)
        assert torch.equal(b.unpack_radon(gb)[i], g1)
        assert torch.equal(b.unpack_data(fb)[i], f1)
        plan.close()
    b.close()


def test_uneven_batch_equals_single_calls():
    run_batch(DESCS, 40)


def test_c4_shaped_batch_equals_single_calls():
    """Eight gathers drawn like the uneven batch workload (nt in {512, 1024,
    2048}, nx in 128..1024)."""
    run_batch(synth.batch_descs(8, seed=4), 60)


@pytest.mark.parametrize("flags", [0, 8 | 32, 16 | 64 | 4])
def test_batch_matches_oracle_every_member_both_directions(flags):
    """Every gather of an uneven batch (four grids, among them a ragged and
    a 16 x 16 one), forward and adjoint, against the FP64 oracle to the
    single-gather bar; also with kernel variants (band heights 4 and 2,
    other chunk sizes, column pairs) that the batch's gathers take."""
    from paper_1604_07651_amd.hrt import Batch
    descs = DESCS[:4]
    b = Batch(descs, flags=flags)
    pairs = [synth.random_pair(d, 70 + i) for i, d in enumerate(descs)]
    print(f"[gpu] batch vs oracle, flags {flags}", flush=True)
    gb = b.forward(b.pack_data([p[0] for p in pairs]))
    fb = b.adjoint(b.pack_radon([p[1] for p in pairs]))
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        ora = logpolar.LogPolarOracle(d)
        for what, got, ref in (("forward", b.unpack_radon(gb)[i], ora.forward(pairs[i][0])),
                               ("adjoint", b.unpack_data(fb)[i], ora.adjoint(pairs[i][1]))):
            got = got.double().cpu().numpy()
            r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            m = np.abs(got - ref).max() / np.abs(ref).max()
            print(f"  member {i} {what}: rel-L2 {r:.2e} max/peak {m:.2e}", flush=True)
            assert r <= 1e-5 and m <= 1e-4
    b.close()


def _ista_inputs(descs, seed):
    from paper_1604_07651_amd.hrt import Batch
    b = Batch(descs)
    fs, masks = [], []
    for i, d in enumerate(descs):
        f, _ = synth.random_pair(d, seed + i, dtype=np.float32)
        keep = synth.trace_mask(d.nx, 0.4, seed + 100 + i)
        m = np.repeat(keep[:, None], d.nt, 1).astype(np.float32)
        fs.append(f * m)
        masks.append(m)
    return b, b.pack_data(fs), b.pack_data(masks)


def test_batch_ista_equals_per_gather_iterations():
    """Soft-thresholding iterations for a whole batch, each gather with its
    own step and weight, equal each gather's own iterations bit for bit."""
    import ctypes as C
    from paper_1604_07651_amd import _lib
    descs = DESCS[:3] + [DESCS[4]]
    b, F, M = _ista_inputs(descs, 70)
    n = len(descs)
    c2 = [0.02, 0.03, 0.015, 0.01]
    mu = [0.5, 0.0, 1.5, 0.2]
    G = torch.zeros(b.radon_off[-1], device="cuda")
    print("[gpu] batch ista", flush=True)
    b.ista_iterate(F, G, 4, c2, mu, mask=M)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        h = C.c_void_p()
        _lib.check(b._lib.hrt_batch_plan(b._h, i, C.byref(h)), "hrt_batch_plan")
        f = b.unpack_data(F)[i].contiguous()
        m = b.unpack_data(M)[i].contiguous()
        g = torch.zeros((d.nq, d.ntau), device="cuda")
        wd = torch.empty((d.nx, d.nt), device="cuda")
        wr = torch.empty((d.nq, d.ntau), device="cuda")
        _lib.check(b._lib.hrt_ista_iterate(h, C.c_void_p(f.data_ptr()), C.c_void_p(m.data_ptr()),
                                           C.c_void_p(g.data_ptr()), C.c_void_p(wd.data_ptr()),
                                           C.c_void_p(wr.data_ptr()), 4, c2[i], mu[i], None),
                   "hrt_ista_iterate")
        torch.cuda.synchronize()
        print(f"  gather {i}", flush=True)
        assert torch.equal(b.unpack_radon(G)[i], g)
    b.close()


def test_batch_ista_graph_replays_match_eager():
    """The batched iterations in one HIP graph: every replay (with eager work
    and synchronisations between replays) equals the eager iterations."""
    descs = [DESCS[0], DESCS[2]]
    b, F, M = _ista_inputs(descs, 90)
    c2, mu = [0.02, 0.025], [0.3, 0.6]
    ref = torch.zeros(b.radon_off[-1], device="cuda")
    print("[gpu] batch ista eager", flush=True)
    b.ista_iterate(F, ref, 3, c2, mu, mask=M)
    G = torch.zeros_like(ref)
    gr = b.ista_graph(F, G, 3, c2, mu, mask=M)
    # a later call with other parameters must not change the graph's
    b.ista_iterate(F, torch.zeros_like(ref), 1, [0.5, 0.5], [9.0, 9.0], mask=M)
    for rep in range(3):
        G.zero_()
        torch.cuda.synchronize()
        print(f"[gpu] batch ista graph replay {rep}", flush=True)
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(G, ref)
        b.forward(F)  # eager work between replays
        torch.cuda.synchronize()
    gr.close()
    from paper_1604_07651_amd import _lib
    with pytest.raises(_lib.HrtError):
        b.ista_iterate(F, G, 1, [0.02, -1.0], [0.3, 0.3], mask=M)
    # each member's operator norm, as its own plan gives it
    from paper_1604_07651_amd.hrt import Plan
    for i, d in enumerate(descs):
        assert b.opnorm2(i, iters=10) == Plan(d).opnorm2(iters=10)
    b.close()


def test_non_finite_member_stays_in_its_gather():
    """A NaN or inf in one gather of a batch makes that gather's output NaN
    everywhere (its own input maximum fails, its spread chunks write NaN
    partials) and leaves the other gathers equal to their single calls."""
    from paper_1604_07651_amd.hrt import Batch, Plan
    descs = DESCS[:3]
    b = Batch(descs)
    pairs = [synth.random_pair(d, 90 + i, dtype=np.float32) for i, d in enumerate(descs)]
    keep = logpolar.LogPolarOracle(descs[1]).geo.keep
    for bad in (float("nan"), float("inf")):
        fs = [p[0].copy() for p in pairs]
        gs = [p[1].copy() for p in pairs]
        fs[1][3, 5] = bad
        gs[1][2, 4] = bad
        print(f"[gpu] batch with {bad} in gather 1", flush=True)
        gb = b.unpack_radon(b.forward(b.pack_data(fs)))
        fb = b.unpack_data(b.adjoint(b.pack_radon(gs)))
        torch.cuda.synchronize()
        assert torch.isnan(gb[1]).all()
        assert torch.isnan(fb[1][torch.from_numpy(keep).cuda()]).all()
        for i in (0, 2):
            plan = Plan(descs[i])
            g1 = plan.forward(torch.from_numpy(fs[i]).cuda())
            f1 = plan.adjoint(torch.from_numpy(gs[i]).cuda())
            torch.cuda.synchronize()
            assert torch.equal(gb[i], g1)
            assert torch.equal(fb[i], f1)
            plan.close()
    b.close()
