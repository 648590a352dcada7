"""Pins for the split transform of the oracle (Section 4, eq. tsplit: the
integral over t cut at intermediate times; Section 5: one cut in time and one
in slowness).  Readings S1-S4 are stated in oracle/split.py."""
import math

import numpy as np
import pytest

import synth
from oracle import direct, geometry, logpolar, split

C1 = synth.config_desc("c1")
ODD = synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                     tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("desc", [ODD, C1])
def test_one_band_per_axis_is_the_plain_transform(desc):
    """With one time band and one slowness band the single part is the whole
    problem: its grid is the description and both directions equal the plain
    oracle's."""
    so = split.SplitOracle(desc, [0, desc.nt], [0, desc.nq])
    (p,) = so.parts
    for k in ("nt", "nx", "ntau", "nq", "q0", "dt", "dx", "x0", "tau0", "dtau", "dq"):
        assert getattr(p.desc, k) == getattr(desc, k), k
    plain = logpolar.LogPolarOracle(desc)
    f, g = synth.random_pair(desc, 3)
    assert np.array_equal(so.forward(f), plain.forward(f))
    assert np.array_equal(so.adjoint(g), plain.adjoint(g))


@pytest.mark.parametrize("desc,te,qe", [
    (ODD, [0, 15, 37], [0, 9, 19]),
    (ODD, [0, 9, 20, 37], [0, 19]),
    (C1, [0, 96, 256], [0, 64, 128]),
])
def test_split_adjoint_is_the_transpose(desc, te, qe):
    """Eq. inner for the sum of parts: <R f, g> = <f, R* g> to 1e-12."""
    so = split.SplitOracle(desc, te, qe)
    f, g = synth.random_pair(desc, 17)
    Rf, Rg = so.forward(f), so.adjoint(g)
    assert abs(np.vdot(Rf, g) - np.vdot(f, Rg)) / (np.linalg.norm(Rf) * np.linalg.norm(g)) < 1e-12


def test_part_grids_worked_example():
    """C1 (dt = 4 ms, x in [0, 2] km over 128 traces, q in [1/4, 1/1.5] s/km
    over 128 rows) cut at sample 64 and at row 64, worked by hand:
    time band [0, 64): last sample t = 0.252 s, nt_p = 66; slowness band 0
    (q0 = 0.25): x_k <= 0.252 / 0.25 = 1.008 km holds for k <= 64 (x_64 =
    1.00787 km), 65 traces plus one = 66; tau_i <= 65 * 4 ms: 66 samples.
    Slowness band 1 (q0 = 0.25 + 64 dq = 0.4600 s/km): x_k <= 0.5478 km for
    k <= 34 (x_34 = 0.5354 km), 35 + 1 = 36 traces.  Time band [64, 256): the whole time axis,
    all traces, all tau."""
    ps = split.parts(C1, [0, 64, 256], [0, 64, 128])
    got = [(p.desc.nt, p.desc.nx, p.desc.ntau, p.desc.nq, p.j_lo, p.j_hi, p.l_lo) for p in ps]
    assert got == [(66, 66, 66, 64, 0, 64, 0), (256, 128, 256, 64, 64, 256, 0),
                   (66, 36, 66, 64, 0, 64, 64), (256, 128, 256, 64, 64, 256, 64)]
    assert abs(ps[2].desc.q0 - (0.25 + 64 * (1 / 1.5 - 0.25) / 127)) < 1e-15


@pytest.mark.parametrize("te,qe", [([0, 64, 256], [0, 64, 128]),
                                   ([0, 32, 96, 256], [0, 40, 80, 128])])
def test_parts_take_in_each_kept_sample_once_per_slowness_band(te, qe):
    """Brute force over samples: within one slowness band, every sample with
    t_j >= q0_band x_k (the band's trapezoid) is taken in by exactly one
    part (in the part's own grid), and no other sample is."""
    ps = split.parts(C1, te, qe)
    n_t = len(te) - 1
    for iq in range(len(qe) - 1):
        count = np.zeros((C1.nx, C1.nt), dtype=int)
        for it in range(n_t):
            p = ps[iq * n_t + it]
            keep = geometry.build(p.desc, (p.j_lo, p.j_hi)).keep
            count[:p.desc.nx, :p.desc.nt] += keep
        q0b = C1.q0 + qe[iq] * C1.dq
        want = np.zeros_like(count)
        for k in range(C1.nx):
            for j in range(C1.nt):
                want[k, j] = 1 if j * C1.dt >= q0b * (C1.x0 + k * C1.dx) else 0
        assert np.array_equal(count, want)


def gaussian_exact(desc, cs, cy, w):
    """Closed form of the transform of a Gaussian in (s, y) of the whole
    grid's rescaling (as in the plain oracle's pins)."""
    T = (desc.nt - 1) * desc.dt
    X = desc.x0 + (desc.nx - 1) * desc.dx
    qh = ((desc.q0 + np.arange(desc.nq) * desc.dq) * X / T)[:, None]
    th = ((desc.tau0 + np.arange(desc.ntau) * desc.dtau) / T)[None, :]
    dist = np.abs(cs - th ** 2 - qh ** 2 * cy) / np.sqrt(1 + qh ** 4)
    return X * math.sqrt(2 * math.pi) * w * np.exp(-dist ** 2 / (2 * w ** 2)) / np.sqrt(1 + qh ** 4)


def test_split_through_an_event_matches_the_closed_form():
    """A smooth Gaussian in (s, y) centred on the cut time (t^ = 0.5 of the
    whole grid, sample 128): the two parts' contributions add up to the
    closed-form transform within 4e-3 (plain: 1.3e-3).  Reading S2's two
    extra samples are needed: without them the Radon samples just after the
    cut lose the interpolation reach of the first part's last sample (2e-2
    measured)."""
    f = synth.gaussian_sy_gather(C1, 0.25, 0.15, 0.05)
    exact = gaussian_exact(C1, 0.25, 0.15, 0.05)
    assert rel(logpolar.LogPolarOracle(C1).forward(f), exact) < 2e-3
    assert rel(split.SplitOracle(C1, [0, 128, 256], [0, 128]).forward(f), exact) < 4e-3


def test_split_reduces_the_small_tau_error_against_direct_summation():
    """Section 5: the plain method's errors against direct summation sit at
    small tau; one cut in time and one in slowness (the paper's set-up)
    reduces them.  On C1 (five 25 Hz Ricker events): the error in the first
    quarter of tau drops at least 2x, the whole panel's by 30 %, and more
    cuts reduce it further."""
    f = synth.config_gather("c1")
    D = direct.forward(C1, f)
    n = np.linalg.norm(D)
    q1 = slice(0, C1.ntau // 4)

    def errs(g):
        return np.linalg.norm((g - D)[:, q1]) / n, rel(g, D)

    e_plain = errs(logpolar.LogPolarOracle(C1).forward(f))
    e_11 = errs(split.SplitOracle(C1, [0, 96, 256], [0, 64, 128]).forward(f))
    e_more = errs(split.SplitOracle(C1, [0, 32, 64, 128, 256], [0, 32, 64, 96, 128]).forward(f))
    assert e_11[0] < 0.5 * e_plain[0]
    assert e_11[1] < 0.7 * e_plain[1]
    assert e_more[1] < 0.75 * e_11[1]


def test_bad_edges_are_rejected():
    with pytest.raises(ValueError):
        split.parts(C1, [0, 100, 90, 256], [0, 128])
    with pytest.raises(ValueError):
        split.parts(C1, [0, 256], [1, 128])
    with pytest.raises(ValueError):
        split.parts(C1, [0, 255], [0, 128])
