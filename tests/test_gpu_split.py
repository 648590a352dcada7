"""GPU parity of the split transform (Section 4, eq. tsplit; Section 5)
through the C ABI against the oracle's split, same tolerances as the plain
transform: rel-L2 <= 1e-5 and max abs error <= 1e-4 of the peak per result,
the float32 dot-product test <= 1e-5."""
import numpy as np
import pytest

import synth
from oracle import split as osplit

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

REL_L2 = 1e-5
MAX_ABS = 1e-4

ODD = synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                     tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5)
RAGGED = synth.GridDesc(nt=301, nx=77, dt=0.004, x0=0.1, dx=0.025, ntau=250, nq=61,
                        tau0=0.05, dtau=0.0045, q0=0.22, dq=0.0075, oversample=2.0)
CASES = {
    "odd_2x2": (ODD, [0, 15, 37], [0, 9, 19]),
    "odd_3x1": (ODD, [0, 9, 20, 37], [0, 19]),
    "c1_paper": (synth.config_desc("c1"), [0, 96, 256], [0, 64, 128]),
    "c1_4x4": (synth.config_desc("c1"), [0, 32, 64, 128, 256], [0, 32, 64, 96, 128]),
    "ragged_2x3": (RAGGED, [0, 120, 301], [0, 20, 41, 61]),
    "c2_paper": (synth.config_desc("c2"), [0, 384, 1024], [0, 256, 512]),
}


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def compare(got, ref, what):
    got = np.asarray(got, dtype=np.float64)
    r = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    m = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {what}: rel-L2 {r:.2e}  max-abs/peak {m:.2e}", flush=True)
    assert r <= REL_L2, f"{what}: rel-L2 {r:.3e}"
    assert m <= MAX_ABS, f"{what}: max abs {m:.3e}"


_cache = {}


def setup(name):
    if name not in _cache:
        from paper_1604_07651_amd.hrt import Split
        desc, te, qe = CASES[name]
        print(f"[split] {name} t {te} q {qe}", flush=True)
        _cache[name] = (desc, Split(desc, te, qe), osplit.SplitOracle(desc, te, qe))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_split_parity(name):
    desc, sp, ora = setup(name)
    f, g = synth.random_pair(desc, 21)
    out = torch.full(sp.radon_shape, float("nan"), device="cuda")
    print(f"[gpu] split forward {name}", flush=True)
    sp.forward(to_gpu(f), out=out)
    torch.cuda.synchronize()
    compare(out.cpu().numpy(), ora.forward(f), f"split forward {name}")
    outa = torch.full(sp.data_shape, float("nan"), device="cuda")
    print(f"[gpu] split adjoint {name}", flush=True)
    sp.adjoint(to_gpu(g), out=outa)
    torch.cuda.synchronize()
    ref = ora.adjoint(g)
    compare(outa.cpu().numpy(), ref, f"split adjoint {name}")
    # samples outside every part's trapezoid are exact zeros
    assert np.all(outa.cpu().numpy()[ref == 0.0] == 0.0)


@pytest.mark.parametrize("name", ["c1_paper", "ragged_2x3", "c2_paper"])
def test_split_dot_product_float32(name):
    desc, sp, ora = setup(name)
    f, g = synth.random_pair(desc, 34)
    F, G = to_gpu(f), to_gpu(g)
    print(f"[gpu] split dot {name}", flush=True)
    Rf = sp.forward(F).double()
    Rg = sp.adjoint(G).double()
    lhs = torch.sum(Rf * G.double()).item()
    rhs = torch.sum(F.double() * Rg).item()
    err = abs(lhs - rhs) / (Rf.norm().item() * G.double().norm().item())
    print(f"  dot test {name}: {err:.2e}", flush=True)
    assert err <= 1e-5


def test_one_band_per_axis_equals_the_plan_bitwise():
    """A split into one part runs the plain plan's kernels on the same
    lists: identical results."""
    from paper_1604_07651_amd.hrt import Plan, Split
    desc = synth.config_desc("c1")
    sp = Split(desc, [0, desc.nt], [0, desc.nq])
    plan = Plan(desc)
    f, g = synth.random_pair(desc, 5)
    print("[gpu] one-part split vs plan", flush=True)
    assert torch.equal(sp.forward(to_gpu(f)), plan.forward(to_gpu(f)))
    assert torch.equal(sp.adjoint(to_gpu(g)), plan.adjoint(to_gpu(g)))


def test_full_size_split_parity():
    """C3 (2048 x 1024 -> 2048 x 1024) with the paper's one cut in time and
    one in slowness: both directions against the oracle's split."""
    from paper_1604_07651_amd.hrt import Split
    desc = synth.config_desc("c3")
    te, qe = [0, 768, 2048], [0, 512, 1024]
    sp = Split(desc, te, qe)
    ora = osplit.SplitOracle(desc, te, qe)
    f = synth.config_gather("c3")
    print("[gpu] split forward c3", flush=True)
    g = sp.forward(to_gpu(f))
    torch.cuda.synchronize()
    g_np = g.cpu().numpy().astype(np.float64)
    compare(g_np, ora.forward(f), "split forward c3")
    print("[gpu] split adjoint c3", flush=True)
    fa = sp.adjoint(g)
    torch.cuda.synchronize()
    compare(fa.cpu().numpy(), ora.adjoint(g_np), "split adjoint c3")


def test_split_argument_errors():
    from paper_1604_07651_amd import _lib
    from paper_1604_07651_amd.hrt import Split
    desc, sp, ora = setup("odd_2x2")
    with pytest.raises(ValueError):
        sp.forward(torch.zeros(sp.radon_shape, device="cuda"))
    with pytest.raises(_lib.HrtError):
        Split(desc, [0, 20, 10, 37], [0, 19])
    with pytest.raises(NotImplementedError):
        sp.opnorm2()
    import ctypes as C
    buf = torch.zeros(desc.nx * desc.nt + 10, device="cuda")
    st = sp._lib.hrt_split_forward(sp._h, C.c_void_p(buf.data_ptr()),
                                   C.c_void_p(buf.data_ptr() + 8), None)
    assert st == 1  # overlapping input and output refused before any launch
