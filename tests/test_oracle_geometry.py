"""Pins for the oracle's geometry (Section 2.1, eqs. transformT/transformP,
Section 2.2 eq. hypnorm, Section 4 eq. lpsamples)."""
import math

import numpy as np
import pytest

import synth
from oracle import geometry


DESCS = [synth.config_desc("c1"), synth.config_desc("c2"),
         synth.GridDesc(nt=64, nx=40, dt=0.01, x0=0.0, dx=0.05, ntau=50,
                        nq=30, tau0=0.1, dtau=0.01, q0=0.3, dq=0.02)]


def test_next_even_smooth():
    assert geometry.next_even_smooth(271) == 288
    assert geometry.next_even_smooth(2160) == 2160
    assert geometry.next_even_smooth(2161) == 2250
    assert geometry.next_even_smooth(7) == 8
    for n in range(2, 400):
        m = geometry.next_even_smooth(n)
        assert m >= n and m % 2 == 0
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        assert r == 1


@pytest.mark.parametrize("desc", DESCS)
def test_square_corners_on_sector_border(desc):
    """Section 2.1: three corners of the square lie on the sector border:
    (0,0) on the -beta/2 ray, (1,1) on the +beta/2 ray, (1,0) on the unit
    arc (readings R2/R3)."""
    g = geometry.build(desc)
    A = geometry.map_T(0.0, 0.0, g.alpha, g.a, g.O1, g.O2)
    B = geometry.map_T(1.0, 0.0, g.alpha, g.a, g.O1, g.O2)
    C = geometry.map_T(1.0, 1.0, g.alpha, g.a, g.O1, g.O2)
    assert abs(math.atan2(A[1], A[0]) + g.beta / 2) < 1e-14
    assert abs(math.atan2(C[1], C[0]) - g.beta / 2) < 1e-14
    assert abs(math.hypot(B[0], B[1]) - 1.0) < 1e-14


def test_printed_O1_is_not_on_the_rays():
    """The O_1 printed in Section 2.1 (with tan beta) misplaces the square;
    this is why reading R2 replaces it."""
    g = geometry.build(synth.config_desc("c2"))
    O1_printed = g.a * math.sin(g.alpha + math.pi / 4) * math.tan(g.beta) / math.sqrt(2)
    A = geometry.map_T(0.0, 0.0, g.alpha, g.a, O1_printed, g.O2)
    assert abs(math.atan2(A[1], A[0]) + g.beta / 2) > 0.1


def test_side_a_is_the_printed_formula_from_the_corner_conditions():
    """Solving |O + a w'| = 1 with O from the two ray conditions gives the
    printed a of Section 2.1; check by bisection on the corner condition."""
    for qmin, qmax in [(0.2, 0.7), (0.5, 1.3), (0.12, 0.33)]:
        alpha, beta, a, O1, O2, _ = geometry.sector(qmin, qmax)

        def corner_B_radius(aa):
            o1 = aa * math.sin(alpha + math.pi / 4) / (math.sqrt(2) * math.tan(beta / 2))
            o2 = aa * math.cos(alpha + math.pi / 4) * math.tan(beta / 2) / math.sqrt(2)
            u, v = geometry.map_T(1.0, 0.0, alpha, aa, o1, o2)
            return math.hypot(u, v) - 1.0

        lo, hi = 1e-6, 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if corner_B_radius(mid) > 0:
                hi = mid
            else:
                lo = mid
        assert abs(lo - a) < 1e-13


@pytest.mark.parametrize("desc", DESCS)
def test_supports_lie_in_the_log_polar_window(desc):
    """Section 2.1: kept data and all outputs lie in
    [-beta/2, beta/2] x [log a_r, 0]; a_r is the smallest output radius
    (attained by the tau = 0, q_min line)."""
    g = geometry.build(desc)
    eps = 1e-13
    assert g.phi[g.keep].min() >= -g.beta / 2 - eps
    assert g.phi[g.keep].max() <= g.beta / 2 + eps
    assert g.eta[g.keep].min() >= math.log(g.a_r) - eps
    assert g.eta[g.keep].max() <= eps
    assert g.rho.min() >= math.log(g.a_r) - eps
    assert g.rho.max() <= eps
    # line through corner A with q = q_min has radius exactly a_r
    d0 = desc.with_(tau0=0.0)
    g0 = geometry.build(d0)
    assert abs(math.exp(g0.rho[0, 0]) - g0.a_r) < 1e-14


@pytest.mark.parametrize("desc", DESCS)
def test_hyperbolas_map_onto_log_polar_lines(desc):
    """Eqs. Rhdef2 + transformT + transformP: the samples of the hyperbola
    t = sqrt(tau^2 + q^2 x^2) land on the line u cos(theta_l) + v sin(theta_l)
    = e^{rho_il} (reading R5)."""
    g = geometry.build(desc)
    rng = np.random.default_rng(0)
    for _ in range(20):
        l = rng.integers(desc.nq)
        i = rng.integers(desc.ntau)
        xh = rng.uniform(0, 1, 16)
        th = np.sqrt(g.tauhat[i] ** 2 + (g.qhat[l] * xh) ** 2)
        u, v = geometry.map_T(th ** 2, xh ** 2, g.alpha, g.a, g.O1, g.O2)
        lhs = u * math.cos(g.theta[l]) + v * math.sin(g.theta[l])
        assert np.abs(lhs - math.exp(g.rho[l, i])).max() < 1e-13


def test_trapezoid_cut_is_where_no_hyperbola_reaches():
    """Section 2.1: no data above t = k x; with k = q_min every hyperbola
    sample has t >= q_min x (reading R4)."""
    d = DESCS[2]
    keep = geometry.kept_mask(d)
    t = np.arange(d.nt) * d.dt
    x = d.x0 + np.arange(d.nx) * d.dx
    assert np.array_equal(keep, t[None, :] >= d.q0 * x[:, None])
    tau = d.tau0 + np.arange(d.ntau) * d.dtau
    q = d.q0 + np.arange(d.nq) * d.dq
    th = np.sqrt(tau[:, None, None] ** 2 + (q[None, :, None] * x[None, None, :]) ** 2)
    assert (th >= d.q0 * x[None, None, :] - 1e-15).all()


@pytest.mark.parametrize("desc", DESCS[:2])
def test_smear_weight_is_the_jacobian_over_2x(desc):
    """Eq. B3tx: the smear weight is f/(2x) e^eta J with J the Jacobian of
    (t, x) -> (phi, eta); reading R8 writes e^eta J/(2x) = 2 a^2 t e^-eta.
    Check against a central-difference Jacobian."""
    g = geometry.build(desc)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(30):
        t = rng.uniform(0.3, 0.95)
        x = rng.uniform(0.05, 0.95) * t / max(g.kslope, 1e-3)
        x = min(x, 0.95)

        def pe(tt, xx):
            u, v = geometry.map_T(tt * tt, xx * xx, g.alpha, g.a, g.O1, g.O2)
            return np.array(geometry.map_P1(u, v))

        dpt = (pe(t + h, x) - pe(t - h, x)) / (2 * h)
        dpx = (pe(t, x + h) - pe(t, x - h)) / (2 * h)
        J = abs(dpt[0] * dpx[1] - dpt[1] * dpx[0])
        eta = pe(t, x)[1]
        lhs = math.exp(eta) * J / (2 * x)
        rhs = 2 * g.a ** 2 * t * math.exp(-eta)
        assert abs(lhs - rhs) < 1e-7 * rhs


@pytest.mark.parametrize("desc", DESCS)
def test_lattice_spacing_and_extent(desc):
    """Eq. lpsamples: the lattice is at least as fine as the largest
    neighbour distance of mapped samples (divided by the oversampling), and
    its periods leave room for the circular convolution not to wrap
    (reading R10)."""
    g = geometry.build(desc)
    keep = g.keep
    dphi = np.abs(np.diff(g.phi, axis=1))[keep[:, 1:] & keep[:, :-1]]
    assert dphi.max() <= g.sigma * g.dtheta * (1 + 1e-15)
    assert g.Ptheta > 2 * g.beta_k
    assert g.Prho > abs(math.log(g.a_r)) + abs(math.log(math.cos(g.beta_k))) + 4 * g.drho
    assert g.Mtheta % 2 == 0 and g.Mrho % 2 == 0


def test_validation_rejects_bad_grids():
    d = DESCS[2]
    for bad in [d.with_(nt=3), d.with_(dq=0.0), d.with_(q0=-0.1),
                d.with_(ntau=100), d.with_(oversample=1.2)]:
        with pytest.raises(ValueError):
            geometry.build(bad)
