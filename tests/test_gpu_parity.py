"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (float32 lattice arithmetic against the float64 oracle of the same
discrete operator): rel-L2 <= 1e-5 per result and max abs error <= 1e-4 of
the reference's peak; the float32 dot-product test <= 1e-5 (the paper's
inner-product test reports O(1e-5) in single precision, Section 5)."""
import numpy as np
import pytest

import synth
from oracle import direct, kernel, logpolar

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
MAX_ABS = 1e-4

SMALL = {
    "c1": synth.config_desc("c1"),
    "odd": synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                          tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5),
    "tiny": synth.GridDesc(nt=16, nx=16, dt=0.01, x0=0.0, dx=0.02, ntau=16, nq=16,
                           tau0=0.0, dtau=0.01, q0=0.25, dq=(1 / 1.5 - 0.25) / 15),
    "ragged": synth.GridDesc(nt=301, nx=77, dt=0.004, x0=0.1, dx=0.025, ntau=250,
                             nq=61, tau0=0.05, dtau=0.0045, q0=0.22, dq=0.0075,
                             oversample=2.0),
    "c2": synth.config_desc("c2"),
    # q0 = 0: the trapezoid keeps every sample
    "q0zero": synth.GridDesc(nt=64, nx=48, dt=0.01, x0=0.0, dx=0.03, ntau=60, nq=40,
                             tau0=0.0, dtau=0.01, q0=0.0, dq=0.008),
    # more traces and slownesses than a band workgroup has threads
    "wide": synth.GridDesc(nt=96, nx=1500, dt=0.004, x0=0.0, dx=4.0 / 1499, ntau=80,
                           nq=1100, tau0=0.0, dtau=0.0048, q0=0.25,
                           dq=(1 / 1.5 - 0.25) / 1099),
    # log-radius axis of 4320 points: longer than the column kernel holds in
    # registers (K read at the multiply) and than its in-place FFT takes
    # (ping-pong passes)
    "long": synth.GridDesc(nt=6000, nx=96, dt=0.0007, x0=0.0, dx=1.5 / 95, ntau=6000,
                           nq=96, tau0=0.0, dtau=0.0007, q0=0.25, dq=(1 / 1.5 - 0.25) / 95),
    # angle axis of 4320 points (the lattice width of the paper's N = 2^11
    # row): the row FFTs take two row pairs through an LDS scratch
    "ang4320": synth.GridDesc(nt=512, nx=2048, dt=0.008, x0=0.0, dx=4.0 / 2047, ntau=512,
                              nq=192, tau0=0.0, dtau=0.008, q0=0.25,
                              dq=(1 / 1.5 - 0.25) / 191),
    # angle axis of 8640 points (the lattice width of the N = 2^12 row): the
    # plan takes bands of 2 rows, one row pair per row-FFT workgroup
    "ang8640": synth.GridDesc(nt=1024, nx=4096, dt=0.004, x0=0.0, dx=4.0 / 4095, ntau=1024,
                              nq=192, tau0=0.0, dtau=0.004, q0=0.25,
                              dq=(1 / 1.5 - 0.25) / 191),
    # the smallest grid the boundary takes (4 samples on every axis), and
    # grids of 4 time samples or 4 traces
    "min4": synth.GridDesc(nt=4, nx=4, dt=0.01, x0=0.0, dx=0.02, ntau=4, nq=4, tau0=0.0,
                           dtau=0.01, q0=0.25, dq=0.1),
    "nt4": synth.GridDesc(nt=4, nx=200, dt=0.1, x0=0.0, dx=0.01, ntau=4, nq=4, tau0=0.0,
                          dtau=0.1, q0=0.25, dq=0.1),
    "nx4": synth.GridDesc(nt=300, nx=4, dt=0.004, x0=0.0, dx=0.5, ntau=300, nq=4, tau0=0.0,
                          dtau=0.004, q0=0.25, dq=0.1),
    # the paper's N = 2^12 grid of the size sweep, whole (dot test only)
    "s4096": synth.s1_desc(4096),
}
# log-radius axes of 256 x R points (R = 2, 3, 4, 5, 8, 9, 10, 15, 16): the
# column pass's last forward radix R, whose outputs the multiply by K takes
# in registers, and whose first pass reads the column from S (C2 and C3
# cover R = 6, 12)
for _name, (_nt, _nx, _X, _qmax, _ov) in {
        "colr2": (400, 48, 1.0, 1 / 1.5, 2.0), "colr3": (1200, 24, 2.0, 1 / 1.5, 2.0),
        "colr4": (1000, 16, 0.5, 1 / 1.5, 2.0), "colr5": (1200, 32, 2.0, 0.5, 2.0),
        "colr8": (2000, 16, 0.5, 1 / 1.5, 2.0), "colr9": (2500, 24, 1.0, 2.0, 3.0),
        "colr10": (2000, 16, 0.5, 1 / 1.5, 2.5), "colr15": (2500, 16, 0.5, 1 / 1.5, 3.0),
        "colr16": (2300, 16, 0.5, 1.0, 3.5)}.items():
    SMALL[_name] = synth.GridDesc(nt=_nt, nx=_nx, dt=0.004, x0=0.0, dx=_X / (_nx - 1), ntau=_nt,
                                  nq=_nx, tau0=0.0, dtau=0.004, q0=0.25,
                                  dq=(_qmax - 0.25) / (_nx - 1), oversample=_ov)

_cache = {}


def setup(name):
    if name not in _cache:
        from paper_1604_07651_amd.hrt import Plan
        desc = SMALL[name] if name in SMALL else synth.config_desc(name)
        print(f"[plan] {name} {desc}", flush=True)
        plan = Plan(desc)
        ora = logpolar.LogPolarOracle(desc)
        _cache[name] = (desc, plan, ora)
    return _cache[name]


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def compare(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    m = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {what}: rel-L2 {r:.2e}  max-abs/peak {m:.2e}", flush=True)
    assert r <= REL_L2, f"{what}: rel-L2 {r:.3e}"
    assert m <= MAX_ABS, f"{what}: max abs {m:.3e}"


@pytest.mark.parametrize("name", ["c1", "odd", "tiny", "ragged"])
def test_kernel_multiplier_matches_oracle(name):
    desc, plan, ora = setup(name)
    K = plan.kernel()
    K1, K2 = K.shape
    ref = ora.K[:K1, :K2]
    assert np.abs(K - ref).max() <= 2e-7 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["c1", "odd", "tiny", "ragged", "q0zero", "wide", "c2",
                                  "long", "ang4320", "ang8640", "min4", "nt4", "nx4",
                                  "colr2", "colr3", "colr4", "colr5", "colr8", "colr9",
                                  "colr10", "colr15", "colr16"])
@pytest.mark.parametrize("kind", ["random", "ricker"])
def test_forward_and_adjoint_parity(name, kind):
    desc, plan, ora = setup(name)
    if kind == "random":
        f, g = synth.random_pair(desc, 21)
    else:
        f = synth.ricker_gather(desc, 12, 20.0, 5)
        g = ora.forward(f)
    # outputs start as NaN: every sample must be written exactly by one band
    print(f"[gpu] forward {name} {kind}", flush=True)
    gf = torch.full(plan.radon_shape, float("nan"), device="cuda")
    plan.forward(to_gpu(f), out=gf)
    torch.cuda.synchronize()
    compare(gf.cpu().numpy(), ora.forward(f), f"forward {name}/{kind}")
    print(f"[gpu] adjoint {name} {kind}", flush=True)
    fa = torch.full(plan.data_shape, float("nan"), device="cuda")
    plan.adjoint(to_gpu(g), out=fa)
    torch.cuda.synchronize()
    ref = ora.adjoint(g)
    got = fa.cpu().numpy()
    compare(got, ref, f"adjoint {name}/{kind}")
    # outside the trapezoid the adjoint is exactly zero
    assert np.all(got[~ora.geo.keep] == 0.0)


def setup_plan_only(name):
    """A plan without the oracle (grids too large for it)."""
    key = ("plan", name)
    if key not in _cache:
        from paper_1604_07651_amd.hrt import Plan
        desc = SMALL[name] if name in SMALL else synth.config_desc(name)
        print(f"[plan] {name}", flush=True)
        _cache[key] = (desc, Plan(desc), None)
    return _cache[key]


@pytest.mark.parametrize("name", ["c1", "ragged", "c2", "min4", "c3", "s4096"])
def test_dot_product_float32(name):
    """The adjoint identity <R f, g> = <f, R* g> in float32 (a property that
    holds at any size, so it also checks the full C3 grid and the N = 2^12
    grid of the size sweep, 8640 x 6250 lattice with 2-row bands, which the
    oracle cannot transform in seconds)."""
    desc, plan, ora = (setup(name) if name not in ("c3", "s4096") else setup_plan_only(name))
    f, g = synth.random_pair(desc, 33)
    F, G = to_gpu(f), to_gpu(g)
    print(f"[gpu] dot {name}", flush=True)
    Rf = plan.forward(F).double()
    Rg = plan.adjoint(G).double()
    lhs = torch.sum(Rf * G.double()).item()
    rhs = torch.sum(F.double() * Rg).item()
    err = abs(lhs - rhs) / (Rf.norm().item() * G.double().norm().item())
    print(f"  dot test {name}: {err:.2e}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("name", ["c3"])
def test_full_size_parity(name):
    """The benchmark workload at full size (2048 x 1024 -> 2048 x 1024, more
    traces and slownesses than one workgroup has threads)."""
    desc, plan, ora = setup(name)
    f = synth.config_gather(name)
    print(f"[gpu] forward {name}", flush=True)
    g = plan.forward(to_gpu(f))
    torch.cuda.synchronize()
    g_np = g.cpu().numpy().astype(np.float64)
    compare(g_np, ora.forward(f), f"forward {name}")
    print(f"[gpu] adjoint {name}", flush=True)
    fa = plan.adjoint(g)
    torch.cuda.synchronize()
    compare(fa.cpu().numpy(), ora.adjoint(g_np), f"adjoint {name}")


@pytest.mark.parametrize("name", ["c1", "ragged", "q0zero", "c2", "long", "c3"])
def test_normal_equals_forward_then_adjoint(name):
    """hrt_normal (the adjoint's input maximum taken from the forward's
    gather) gives exactly the two separate calls, also with fa over f."""
    desc, plan, ora = setup(name)
    f = to_gpu(synth.random_pair(desc, 31)[0])
    print(f"[gpu] normal {name}", flush=True)
    g1 = plan.forward(f)
    fa1 = plan.adjoint(g1)
    g2, fa2 = plan.normal(f)
    f3 = f.clone()
    g3, fa3 = plan.normal(f3, out=f3)
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(fa1, fa2)
    assert torch.equal(g1, g3) and torch.equal(fa1, fa3)


def test_normal_non_finite_zero_and_overlap():
    from paper_1604_07651_amd import _lib
    desc, plan, ora = setup("c1")
    print("[gpu] normal: zero, non-finite, overlap", flush=True)
    f = np.zeros((desc.nx, desc.nt), dtype=np.float32)
    g, fa = plan.normal(to_gpu(f))
    torch.cuda.synchronize()
    assert not g.any() and not fa.any()
    f[3, 100] = np.inf
    g, fa = plan.normal(to_gpu(f))
    torch.cuda.synchronize()
    assert torch.isnan(g).all()
    assert torch.isnan(fa[torch.from_numpy(ora.geo.keep).cuda()]).all()
    # g overlapping f is refused before anything is launched
    nd, nr = desc.nx * desc.nt, desc.nq * desc.ntau
    buf = torch.zeros(nd + nr, device="cuda")
    fv = buf[:nd].view(desc.nx, desc.nt)
    gv = buf[nd - 8:nd - 8 + nr].view(desc.nq, desc.ntau)
    with pytest.raises(_lib.HrtError):
        plan.normal(fv, g=gv)


def test_non_finite_input_gives_nan_everywhere():
    """One NaN or inf in the input makes the whole output NaN (the spread's
    fixed-point scale cannot be formed), in both directions."""
    desc, plan, ora = setup("c1")
    f, g = synth.random_pair(desc, 8)
    print("[gpu] non-finite inputs", flush=True)
    for bad in (float("nan"), float("inf")):
        F = to_gpu(f)
        F[3, 100] = bad
        assert torch.isnan(plan.forward(F)).all()
        G = to_gpu(g)
        G[5, 7] = bad
        out = plan.adjoint(G)
        assert torch.isnan(out[torch.from_numpy(ora.geo.keep).cuda()]).all()
    # a finite input afterwards is unaffected
    compare(plan.forward(to_gpu(f)).cpu().numpy(), ora.forward(f), "forward after NaN")


def test_zero_input_gives_zero_output():
    desc, plan, ora = setup("c1")
    z = torch.zeros(plan.data_shape, device="cuda")
    print("[gpu] zeros", flush=True)
    assert torch.count_nonzero(plan.forward(z)).item() == 0
    zr = torch.zeros(plan.radon_shape, device="cuda")
    assert torch.count_nonzero(plan.adjoint(zr)).item() == 0


def test_outputs_are_overwritten_and_stream_respected():
    desc, plan, ora = setup("c1")
    f, g = synth.random_pair(desc, 3)
    F = to_gpu(f)
    out = torch.full(plan.radon_shape, float("nan"), device="cuda")
    s = torch.cuda.Stream()
    print("[gpu] side stream", flush=True)
    with torch.cuda.stream(s):
        plan.forward(F, out=out)
    s.synchronize()
    ref = plan.forward(F)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
    assert torch.allclose(out, ref, rtol=1e-6, atol=1e-6 * ref.abs().max().item())


def test_argument_errors():
    desc, plan, ora = setup("odd")
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(plan.radon_shape, device="cuda"))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(plan.data_shape, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        plan.forward(torch.zeros(plan.data_shape))
    from paper_1604_07651_amd import _lib
    import ctypes as C
    buf = torch.zeros(plan.data_shape[0] * plan.data_shape[1] + 10, device="cuda")
    st = plan._lib.hrt_forward(plan._h, C.c_void_p(buf.data_ptr()),
                               C.c_void_p(buf.data_ptr() + 8), None)
    assert st == 1  # overlapping input and output refused before any launch


def test_direct_sum_matches_oracle():
    desc, plan, ora = setup("c1")
    f, g = synth.random_pair(desc, 8)
    print("[gpu] direct c1", flush=True)
    got = plan.direct_forward(to_gpu(f))
    torch.cuda.synchronize()
    ref = direct.forward(desc, f)
    r = np.linalg.norm(got.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  direct forward rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-4
    gota = plan.direct_adjoint(to_gpu(g))
    torch.cuda.synchronize()
    refa = direct.adjoint(desc, g)
    r = np.linalg.norm(gota.cpu().numpy() - refa) / np.linalg.norm(refa)
    print(f"  direct adjoint rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-4
    # float32 transpose identity of the GPU direct sum
    F, G = to_gpu(f), to_gpu(g)
    lhs = torch.sum(plan.direct_forward(F).double() * G.double()).item()
    rhs = torch.sum(F.double() * plan.direct_adjoint(G).double()).item()
    assert abs(lhs - rhs) / abs(lhs) <= 1e-5


# direct-sum grids: offsets in time and space, a tau step of 3.75 time
# samples (one tau moves the taps by several samples), and a panel row too
# long for the adjoint's LDS staging (4 (5 ntau + 2 nt + 4) bytes > 160 KiB:
# the per-sample search kernel; many taus on a short trace, since the
# float32 hyperbola times of long traces, good to c 2^-24 samples, hold the
# direct forward of white noise near 1e-4 of the float64 one already at
# 2048 samples)
DIRECT_GRIDS = {
    "odd": SMALL["odd"],
    "ragged": SMALL["ragged"],
    "coarse_tau": synth.GridDesc(nt=400, nx=40, dt=0.002, x0=0.1, dx=0.05, ntau=100, nq=30,
                                 tau0=0.05, dtau=0.0075, q0=0.2, dq=0.015),
    "many_taus": synth.GridDesc(nt=512, nx=6, dt=0.002, x0=0.0, dx=0.3, ntau=20000, nq=6,
                                tau0=0.0, dtau=511 * 0.002 / 19999, q0=0.25, dq=0.08),
}


@pytest.mark.parametrize("name", list(DIRECT_GRIDS))
def test_direct_sum_paths_match_oracle(name):
    """Both directions of the GPU direct sum against the oracle's, the
    float32 transpose identity between them, and a repeated adjoint bit for
    bit the same (its sums run in a fixed order)."""
    from paper_1604_07651_amd.hrt import Plan
    desc = DIRECT_GRIDS[name]
    staged = 4 * (5 * desc.ntau + 2 * desc.nt + 4) <= 163840
    print(f"[plan] direct {name} (adjoint {'staged rows' if staged else 'search'})", flush=True)
    plan = Plan(desc)
    f, g = synth.random_pair(desc, 44)
    F, G = to_gpu(f), to_gpu(g)
    print(f"[gpu] direct {name}", flush=True)
    got = plan.direct_forward(F)
    gota = plan.direct_adjoint(G)
    gotb = plan.direct_adjoint(G)
    torch.cuda.synchronize()
    assert torch.equal(gota, gotb)
    for what, y, ref in (("forward", got, direct.forward(desc, f)),
                         ("adjoint", gota, direct.adjoint(desc, g))):
        y = y.double().cpu().numpy()
        r = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        print(f"  direct {what} rel-L2 {r:.2e}", flush=True)
        assert r <= 1e-4
    lhs = torch.sum(got.double() * G.double()).item()
    rhs = torch.sum(F.double() * gota.double()).item()
    err = abs(lhs - rhs) / (got.double().norm().item() * G.double().norm().item())
    print(f"  direct transpose identity {err:.2e}", flush=True)
    assert err <= 1e-5
    plan.close()


def test_direct_sum_matches_oracle_c2():
    """The GPU direct sum (the reference the metric compares against) at C2:
    forward on a sample of 16 slowness rows, adjoint of a panel whose only
    non-zero rows are a block of 16 slownesses (the oracle's adjoint of the
    same block as a grid of its own)."""
    desc, plan, ora = setup("c2")
    f, g = synth.random_pair(desc, 12)
    rows = np.arange(0, desc.nq, desc.nq // 16)
    print("[gpu] direct c2", flush=True)
    got = plan.direct_forward(to_gpu(f)).double().cpu().numpy()[rows]
    ref = direct.forward(desc, f, rows=rows)
    r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  direct forward rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-4
    l0, n = 200, 16
    gb = np.zeros_like(g)
    gb[l0:l0 + n] = g[l0:l0 + n]
    gota = plan.direct_adjoint(to_gpu(gb)).double().cpu().numpy()
    sub = desc.with_(nq=n, q0=desc.q0 + l0 * desc.dq)
    refa = direct.adjoint(sub, g[l0:l0 + n])
    r = np.linalg.norm(gota - refa) / np.linalg.norm(refa)
    print(f"  direct adjoint rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-4


def test_log_polar_vs_direct_sum_band_limited_c3():
    """Method accuracy at the benchmark's size: the GPU log-polar forward of
    a band-limited C3 gather (late hyperbolic Ricker events of 30 Hz, edges
    tapered) against the FP64 direct sum on 25 slowness rows, <= 1e-3."""
    desc, plan, ora = setup("c3")
    f = synth.band_limited_gather(desc, 20, 30.0, 7)
    rows = np.arange(0, desc.nq, desc.nq // 24)
    print("[gpu] band-limited c3 vs direct sum", flush=True)
    lp = plan.forward(to_gpu(f)).double().cpu().numpy()[rows]
    ds = direct.forward(desc, f, rows=rows)
    r = np.linalg.norm(lp - ds) / np.linalg.norm(ds)
    print(f"  LP(GPU) vs DS(FP64) rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-3


def test_log_polar_agrees_with_direct_sum_on_band_limited_data():
    """Method accuracy on the GPU: a smooth Gaussian in (s, y) at C1."""
    desc, plan, ora = setup("c1")
    f = synth.gaussian_sy_gather(desc, 0.5, 0.35, 0.05)
    F = to_gpu(f)
    lp = plan.forward(F).double().cpu().numpy()
    ds = direct.forward(desc, f)
    r = np.linalg.norm(lp - ds) / np.linalg.norm(ds)
    print(f"  LP(GPU) vs DS(FP64) rel-L2 {r:.2e}", flush=True)
    assert r <= 1e-3


def test_unaligned_input_matches_aligned():
    """An input that starts 4 bytes past a 16-byte boundary takes the scalar
    path of the input maximum; the result must not change."""
    desc, plan, ora = setup("ragged")
    f, g = synth.random_pair(desc, 5)
    n = f.size
    buf = torch.zeros(n + 1, device="cuda")
    buf[1:] = torch.from_numpy(f.astype(np.float32).ravel()).cuda()
    F_off = buf[1:].view(plan.data_shape)
    assert F_off.data_ptr() % 16 != 0
    print("[gpu] unaligned input", flush=True)
    a = plan.forward(F_off)
    b = plan.forward(F_off.clone())
    torch.cuda.synchronize()
    assert torch.equal(a, b)


# every HRT_TUNE_* bit, alone and in combinations: smaller FFT radices,
# column pairs, band heights 4 and 2, smaller spread chunks, larger gather
# chunks
VARIANT_FLAGS = list(range(1, 8)) + [8, 16, 32, 64, 8 | 32, 16 | 64, 16 | 4 | 32, 8 | 3 | 64]


# (the FFT-only variants, flags below 8, on the ragged grid only)
VARIANT_CASES = ([("ragged", fl) for fl in VARIANT_FLAGS]
                 + [("c2", fl) for fl in VARIANT_FLAGS if fl >= 8])


@pytest.mark.parametrize("name,flags", VARIANT_CASES)
def test_kernel_variants_match_oracle(name, flags):
    """Every kernel variant against the oracle, to the same bar as the
    default; the plan's band height is the one the flags ask for."""
    from paper_1604_07651_amd.hrt import Plan
    desc, _, ora = setup(name)
    plan = Plan(desc, flags=flags)
    want_rows = 2 if flags & 16 else 4 if flags & 8 else 8
    assert plan.info["band_rows"] == want_rows
    f, g = synth.random_pair(desc, 90 + flags)
    print(f"[gpu] variant {name} {flags}", flush=True)
    compare(plan.forward(to_gpu(f)).cpu().numpy(), ora.forward(f), f"forward flags {flags}")
    compare(plan.adjoint(to_gpu(g)).cpu().numpy(), ora.adjoint(g), f"adjoint flags {flags}")
    plan.close()


def test_autotuner_caches_and_plans_use_it(tmp_path, monkeypatch):
    """The coordinate search over the variant dimensions times every option
    of each dimension, picks the fastest it timed, caches it; plans and
    batches created with tuned=True take it."""
    from paper_1604_07651_amd import autotune
    from paper_1604_07651_amd.hrt import Batch, Plan
    monkeypatch.setenv("HRT_TUNE_CACHE", str(tmp_path / "tune.json"))
    desc = SMALL["c1"]
    print("[gpu] autotune c1", flush=True)
    res = autotune.tune(desc, reps=3)
    timed = {int(k) for k in res["ms"]}
    for _, options in autotune.DIMENSIONS:
        mask = 0
        for o in options:
            mask |= o
        # every option of every dimension was timed with the others at some value
        assert all(any((fl & mask) == o for fl in timed) for o in options)
    assert res["flags"] == min(timed, key=lambda f: res["ms"][str(f)])
    assert autotune.tuned_flags(desc) == res["flags"]
    plan = Plan(desc, tuned=True)
    assert plan.flags == res["flags"]
    plan.close()
    b = Batch([desc, SMALL["odd"]], tuned=True)
    assert b.flags == [res["flags"], 0]
    b.close()
    # an explicit list of variants is timed exactly
    res2 = autotune.tune(desc, reps=2, variants=[0, 8, 16], save=False)
    assert set(res2["ms"]) == {"0", "8", "16"}
    # a batch is tuned as a whole, one variant for all its gathers
    descs = [desc, SMALL["odd"], SMALL["ragged"]]
    res3 = autotune.tune_batch(descs, reps=2)
    assert res3["flags"] == min((int(k) for k in res3["ms"]), key=lambda f: res3["ms"][str(f)])
    assert autotune.batch_flags(descs) == res3["flags"]
    assert autotune.batch_flags(descs[:2]) == 0  # another batch: not tuned
