"""GPU parity on seeded random grids: sizes, steps, offsets and oversampling
drawn at random (every axis ragged against the kernels' tiles), forward and
adjoint through the C ABI against the FP64 oracle, at the tolerances of the
fixed-grid parity tests (rel-L2 <= 1e-5, max abs error <= 1e-4 of the
reference's peak).  A grid the plan rejects is drawn again; lattices above
4 M cells are skipped so that the oracle finishes each case in seconds.
Uneven batches of such grids (every member, both directions, with kernel
variants that all members take), and such grids cut at random into time and
slowness bands (against the oracle's split), meet the same bars; so do the
soft-thresholding iterations (half the traces masked) and the multiple
attenuation on random grids, against the oracle's."""
import numpy as np
import pytest

import synth
from oracle import demultiple as odemultiple
from oracle import ista as oista
from oracle import logpolar
from oracle import split as osplit

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
MAX_ABS = 1e-4
N_GRIDS = 32
MAX_CELLS = 4_000_000


def draw_grids(seed=2026, n=N_GRIDS, max_cells=MAX_CELLS, max_samples=None):
    """Seeded random grids that the plan accepts (host-only check)."""
    from paper_1604_07651_amd import hrt
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        nt = int(rng.integers(8, 2500))
        nx = int(rng.integers(4, 700))
        dt = float(rng.choice([0.002, 0.004, 0.008]))
        x0 = float(rng.choice([0.0, round(float(rng.uniform(0.0, 0.3)), 3)]))
        X = float(round(rng.uniform(0.2, 4.0), 3))
        if X <= x0 + 0.05:
            continue
        T = (nt - 1) * dt
        ntau = int(rng.integers(4, 2500))
        tau0 = float(rng.choice([0.0, round(float(rng.uniform(0.0, 0.2 * T)), 4)]))
        dtau = (T - tau0) / (ntau - 1) * float(rng.uniform(0.5, 1.0))
        nq = int(rng.integers(4, 700))
        q0 = float(round(rng.uniform(0.0, 0.4), 3))
        qmax = float(round(rng.uniform(q0 + 0.05, 1.0), 3))
        ov = float(rng.choice([1.5, 2.0, 2.5, 3.0]))
        d = synth.GridDesc(nt=nt, nx=nx, dt=dt, x0=x0, dx=(X - x0) / (nx - 1), ntau=ntau,
                           nq=nq, tau0=tau0, dtau=dtau, q0=q0, dq=(qmax - q0) / (nq - 1),
                           oversample=ov)
        try:
            info = hrt.describe(d)
        except Exception:
            continue
        if info["m_theta"] * info["m_rho"] > max_cells:
            continue
        if max_samples and nt * nx + ntau * nq > max_samples:
            continue
        out.append(d)
    return out


_grids = []


def grid(i):
    if not _grids:
        _grids.extend(draw_grids())
    return _grids[i]


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def compare(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    m = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {what}: rel-L2 {r:.2e}  max-abs/peak {m:.2e}", flush=True)
    assert r <= REL_L2, f"{what}: rel-L2 {r:.3e}"
    assert m <= MAX_ABS, f"{what}: max abs {m:.3e}"


@pytest.mark.parametrize("i", range(N_GRIDS))
def test_random_grid_parity(i):
    from paper_1604_07651_amd.hrt import Plan
    desc = grid(i)
    print(f"[plan] random grid {i}: {desc}", flush=True)
    plan = Plan(desc)
    ora = logpolar.LogPolarOracle(desc)
    f, g = synth.random_pair(desc, 100 + i)
    print(f"[gpu] forward random grid {i}", flush=True)
    gf = torch.full(plan.radon_shape, float("nan"), device="cuda")
    plan.forward(to_gpu(f), out=gf)
    torch.cuda.synchronize()
    compare(gf.cpu().numpy(), ora.forward(f), f"forward grid {i}")
    print(f"[gpu] adjoint random grid {i}", flush=True)
    fa = torch.full(plan.data_shape, float("nan"), device="cuda")
    plan.adjoint(to_gpu(g), out=fa)
    torch.cuda.synchronize()
    got = fa.cpu().numpy()
    compare(got, ora.adjoint(g), f"adjoint grid {i}")
    assert np.all(got[~ora.geo.keep] == 0.0)
    plan.close()


@pytest.mark.parametrize("flags", [0, 8 | 32, 16 | 64])
def test_random_batch_parity(flags):
    from paper_1604_07651_amd.hrt import Batch
    descs = draw_grids(seed=7 + flags, n=6, max_cells=1_500_000)
    b = Batch(descs, flags=flags)
    pairs = [synth.random_pair(d, 200 + i) for i, d in enumerate(descs)]
    print(f"[gpu] random batch of {len(descs)}, flags {flags}", flush=True)
    gb = b.forward(b.pack_data([p[0] for p in pairs]))
    fb = b.adjoint(b.pack_radon([p[1] for p in pairs]))
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        ora = logpolar.LogPolarOracle(d)
        compare(b.unpack_radon(gb)[i].cpu().numpy(), ora.forward(pairs[i][0]),
                f"batch member {i} forward")
        compare(b.unpack_data(fb)[i].cpu().numpy(), ora.adjoint(pairs[i][1]),
                f"batch member {i} adjoint")
    b.close()


def draw_splits(seed=11, n=6):
    """Seeded random grids with random cuts in time and slowness (one to three
    bands per axis), every part accepted by the plan (host-only check)."""
    from paper_1604_07651_amd import hrt
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        d = draw_grids(seed=int(rng.integers(1 << 30)), n=1, max_cells=1_000_000)[0]

        def edges(m, bands):
            cuts = sorted(rng.choice(np.arange(8, m - 7), size=bands - 1, replace=False).tolist()) \
                if m > 16 + 8 * bands else []
            return [0] + [int(c) for c in cuts] + [m]
        te = edges(d.nt, int(rng.integers(1, 4)))
        qe = edges(d.nq, int(rng.integers(1, 4)))
        if np.min(np.diff(te)) < 8 or np.min(np.diff(qe)) < 8:
            continue
        try:
            for part in range((len(te) - 1) * (len(qe) - 1)):
                hrt.describe_part(d, te, qe, part)
        except Exception:
            continue
        out.append((d, te, qe))
    return out


@pytest.mark.parametrize("i", range(6))
def test_random_split_parity(i):
    from paper_1604_07651_amd.hrt import Split
    desc, te, qe = draw_splits()[i]
    print(f"[split] random {i}: {desc} t {te} q {qe}", flush=True)
    sp = Split(desc, te, qe)
    ora = osplit.SplitOracle(desc, te, qe)
    f, g = synth.random_pair(desc, 300 + i)
    print(f"[gpu] split forward random {i}", flush=True)
    out = torch.full(sp.radon_shape, float("nan"), device="cuda")
    sp.forward(to_gpu(f), out=out)
    torch.cuda.synchronize()
    compare(out.cpu().numpy(), ora.forward(f), f"split forward {i}")
    print(f"[gpu] split adjoint random {i}", flush=True)
    outa = torch.full(sp.data_shape, float("nan"), device="cuda")
    sp.adjoint(to_gpu(g), out=outa)
    torch.cuda.synchronize()
    ref = ora.adjoint(g)
    got = outa.cpu().numpy()
    compare(got, ref, f"split adjoint {i}")
    assert np.all(got[ref == 0.0] == 0.0)
    sp.close()


@pytest.mark.parametrize("i", range(3))
def test_random_grid_ista_and_demultiple(i):
    """Twelve soft-thresholding iterations with half the traces masked (eq.
    itersmd), and the multiple attenuation (mute above a sloping border,
    adjoint, subtract), on random grids against the float64 oracle."""
    from paper_1604_07651_amd.hrt import Plan
    desc = draw_grids(seed=31 + i, n=1, max_cells=200_000, max_samples=150_000)[0]
    print(f"[plan] random ista/demultiple {i}: {desc}", flush=True)
    plan = Plan(desc)
    ora = logpolar.LogPolarOracle(desc)
    f, g = synth.random_pair(desc, 400 + i)
    keep = synth.trace_mask(desc.nx, 0.5, 500 + i)
    mask = np.repeat(keep[:, None], desc.nt, axis=1).astype(np.float64)
    f = f * mask
    lam = oista.power_norm2(ora.forward, ora.adjoint, plan.data_shape, iters=40, seed=3)
    c2 = 0.99 / lam
    mu = 0.05 * np.abs(ora.forward(f)).max()
    ref = oista.ista(ora.forward, ora.adjoint, f, 12, c2, mu, mask)
    gg = torch.zeros(plan.radon_shape, device="cuda")
    print(f"[gpu] ista random {i}", flush=True)
    plan.ista_iterate(to_gpu(f), gg, 12, c2, mu, mask=to_gpu(mask))
    torch.cuda.synchronize()
    got = gg.cpu().numpy().astype(np.float64)
    r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  ista rel-L2 {r:.2e}", flush=True)
    assert r <= 2e-5
    qb0 = desc.q0 + 0.5 * (desc.nq - 1) * desc.dq
    slope = 0.05
    print(f"[gpu] demultiple random {i}", flush=True)
    out = plan.demultiple(to_gpu(f), to_gpu(g), qb0, slope)
    torch.cuda.synchronize()
    refd = odemultiple.demultiple(ora.adjoint, desc, f, g, qb0, slope)
    r = np.linalg.norm(out.cpu().numpy().astype(np.float64) - refd) / np.linalg.norm(refd)
    print(f"  demultiple rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-5
    # the part removed on its own (a zero gather: the output is minus the
    # adjoint of the muted panel, with no float32 subtraction hiding it)
    zero = np.zeros_like(f)
    out0 = plan.demultiple(to_gpu(zero), to_gpu(g), qb0, slope)
    torch.cuda.synchronize()
    ref0 = odemultiple.demultiple(ora.adjoint, desc, zero, g, qb0, slope)
    r = np.linalg.norm(out0.cpu().numpy().astype(np.float64) - ref0) / np.linalg.norm(ref0)
    print(f"  demultiple removed part rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-5
    plan.close()
