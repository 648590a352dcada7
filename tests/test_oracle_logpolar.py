"""Pins for the log-polar oracle (Sections 2.1-2.2, Section 3 eq. inner) and
the direct-summation oracle (eq. Rhdef, Section 5)."""
import math

import numpy as np
import pytest

import synth
from oracle import bspline, direct, geometry, logpolar

TINY = synth.GridDesc(nt=16, nx=16, dt=0.01, x0=0.0, dx=0.02, ntau=16, nq=16,
                      tau0=0.0, dtau=0.01, q0=0.25, dq=(1 / 1.5 - 0.25) / 15)
ODD = synth.GridDesc(nt=37, nx=23, dt=0.01, x0=0.05, dx=0.03, ntau=29, nq=19,
                     tau0=0.07, dtau=0.01, q0=0.3, dq=0.021, oversample=2.5)


@pytest.fixture(scope="module")
def op_c1():
    return logpolar.LogPolarOracle(synth.config_desc("c1"))


def gaussian_exact(geo, cs, cy, w):
    """Closed form: f~ is an isotropic Gaussian in (s, y), so its integral
    along s - q^2 y = tau^2 is sqrt(2 pi) w exp(-d^2/(2 w^2)) / sqrt(1+q^4),
    d the distance of the line from the centre; times X (eq. hypnorm)."""
    qh = geo.qhat[:, None]
    th = geo.tauhat[None, :]
    dist = np.abs(cs - th ** 2 - qh ** 2 * cy) / np.sqrt(1 + qh ** 4)
    return geo.X * math.sqrt(2 * math.pi) * w * np.exp(-dist ** 2 / (2 * w ** 2)) / np.sqrt(1 + qh ** 4)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("desc", [TINY, ODD, synth.config_desc("c1")])
def test_dot_product_identity(desc):
    """Eq. inner: <R f, g> = <f, R* g> to 1e-12 for both oracles."""
    op = logpolar.LogPolarOracle(desc)
    f, g = synth.random_pair(desc, 11)
    Rf = op.forward(f)
    Rg = op.adjoint(g)
    assert abs(np.vdot(Rf, g) - np.vdot(f, Rg)) / (np.linalg.norm(Rf) * np.linalg.norm(g)) < 1e-12
    if desc.nt <= 64:
        Df = direct.forward(desc, f)
        Dg = direct.adjoint(desc, g)
        assert abs(np.vdot(Df, g) - np.vdot(f, Dg)) / (np.linalg.norm(Df) * np.linalg.norm(g)) < 1e-12


def test_gaussian_closed_form(op_c1):
    """The whole chain (rescaling, square placement, W, X cos(psi)/a,
    one-sided integral) against the closed-form transform of a Gaussian in
    (s, y) (readings R1, R2, R7, R8)."""
    d = op_c1.desc
    f = synth.gaussian_sy_gather(d, 0.6, 0.3, 0.06)
    exact = gaussian_exact(op_c1.geo, 0.6, 0.3, 0.06)
    assert rel(op_c1.forward(f), exact) < 1e-3
    assert rel(direct.forward(d, f), exact) < 2e-5


def test_gaussian_closed_form_two_sided_reading_fails(op_c1):
    """A factor 2 (the two-sided eq. Rhdef2) would be caught."""
    d = op_c1.desc
    f = synth.gaussian_sy_gather(d, 0.6, 0.3, 0.06)
    exact = gaussian_exact(op_c1.geo, 0.6, 0.3, 0.06)
    assert rel(2 * op_c1.forward(f), exact) > 0.5


def test_log_polar_agrees_with_direct_sum_on_band_limited_data(op_c1):
    """Section 5: the method approximates direct summation; on data that the
    lattice resolves (a smooth Gaussian in (s, y)) the two agree to 1e-3."""
    d = op_c1.desc
    f = synth.gaussian_sy_gather(d, 0.5, 0.35, 0.05)
    assert rel(op_c1.forward(f), direct.forward(d, f)) < 1e-3


def test_log_polar_agrees_with_direct_sum_on_band_limited_ricker_c2():
    """Section 5's comparison on hyperbolic Ricker events that a single part
    represents (late events, tau from 0.7 T; 15 Hz; edges tapered; offsets
    not aliased): LP and DS agree to 1e-3 on a sample of 25 slowness rows
    (measured 7.2e-4; 2.2e-4 at 10 Hz).  A dropped B-spline division or a
    wrong output factor moves this far above the bar."""
    d = synth.config_desc("c2")
    op = logpolar.LogPolarOracle(d)
    f = synth.band_limited_gather(d, 20, 15.0, 7)
    rows = np.arange(0, d.nq, d.nq // 24)
    lp = op.forward(f)[rows]
    ds = direct.forward(d, f, rows=rows)
    assert rel(lp, ds) < 1e-3


def test_kernel_deconvolution_pinned_by_narrow_gaussian():
    """Section 2.2, eqs. d and B3tauq: the kernel multiplier divides the
    kernel spectrum by the squared B-spline transform along each axis (once
    for the smearing, once for the interpolation).  A narrow Gaussian in
    (s, y) on the C2 grid carries enough high lattice frequencies that the
    whole chain matches its closed form to 1e-5 only with both divisions
    right: measured 3.1e-6 here; dividing by b instead of b^2 along the angle
    axis gives 6.3e-5, along the log radius 5.2e-4."""
    d = synth.config_desc("c2")
    op = logpolar.LogPolarOracle(d)
    f = synth.gaussian_sy_gather(d, 0.6, 0.3, 0.015)
    exact = gaussian_exact(op.geo, 0.6, 0.3, 0.015)
    assert rel(op.forward(f), exact) < 1e-5


def test_log_polar_agrees_with_direct_sum_at_the_last_trace(op_c1):
    """Section 2.2, eq. B3tx2 (trapezoid rule in offset): a smooth Gaussian
    in (s, y) centred on the last trace (y = 1) is cut by the record's edge,
    where the trapezoid weight 1/2 of the last trace decides the sum.  The
    method agrees with direct summation to 1e-3 (measured 5.9e-4); a weight of
    1 on the last trace (or on both end traces) gives 4.6e-2."""
    d = op_c1.desc
    f = synth.gaussian_sy_gather(d, 0.6, 0.95, 0.05)
    assert rel(op_c1.forward(f), direct.forward(d, f)) < 1e-3


def _ramp(z):
    """C-infinity step: 0 for z <= 0, 1 for z >= 1."""
    z = np.clip(z, 1e-9, 1.0 - 1e-9)
    a = np.exp(-1.0 / z)
    b = np.exp(-1.0 / (1.0 - z))
    return a / (a + b)


def _mass_test_data(th, xh, k, m=0.05, width=0.15):
    """Smooth data that vanish near the trapezoid's slanted edge t^ = k x^
    and not at the other three edges x^ = 0, x^ = 1, t^ = 1."""
    u = (th - k * xh - m) / width
    h = np.where(u <= 0.0, 0.0, np.where(u >= 1.0, 1.0, _ramp(u)))
    return h * (1.0 + 0.5 * xh + 0.3 * th)


def test_lattice_mass_is_the_trapezoid_quadrature(op_c1):
    """Section 2.2, eq. B3tx2: the smear weights are a quadrature of the
    polar-coordinate integral of eq. lpfwd.  B-splines form a partition of
    unity, so the lattice's total mass after the spread is sum_p W_p f_p; for
    smooth data it must approximate, with the second-order error of the
    trapezoid rule, the integral of f~(s, y) e^(-rho) over the plane of the
    square (f~ = f / (2 sqrt y), eq. f; e^(-rho) = 1/|p|; dp = a^2 ds dy
    because T is a rotation scaled by a), evaluated here by adaptive
    quadrature in (s, y).  Measured 2.8e-6 relative.  Planted in the weights:
    weight 1 on the first trace (x = 0) 3.5e-3, on the last trace 4.0e-3, on
    the last time sample 4.2e-3."""
    from scipy import integrate

    d = op_c1.desc
    g = op_c1.geo
    k = g.qhat[0]
    th = np.arange(d.nt) * d.dt / g.T
    xh = (d.x0 + np.arange(d.nx) * d.dx) / g.X
    f = _mass_test_data(th[None, :], xh[:, None], k)
    M1, M2 = op_c1.lattice_shape
    mass = logpolar.spread(op_c1.d_x, op_c1.d_y, op_c1.d_w * f[op_c1.kept], M1, M2).sum()

    def inner(y):
        xs = math.sqrt(y)

        def fs(s):
            u, v = geometry.map_T(np.array(s), np.array(y), g.alpha, g.a, g.O1, g.O2)
            return float(_mass_test_data(math.sqrt(s), xs, k)) * g.a ** 2 / math.hypot(float(u), float(v))

        s_lo = (k * xs + 0.05) ** 2
        s_mid = min(1.0, (k * xs + 0.2) ** 2)
        val = integrate.quad(fs, s_lo, s_mid, epsabs=0, epsrel=1e-12, limit=200)[0]
        if s_mid < 1.0:
            val += integrate.quad(fs, s_mid, 1.0, epsabs=0, epsrel=1e-12, limit=200)[0]
        return 0.5 * val  # f~ = f / (2 sqrt y); the 1/sqrt(y) is quad's weight

    exact = integrate.quad(inner, 0.0, 1.0, weight="alg", wvar=(-0.5, 0.0),
                           epsabs=0, epsrel=1e-11, limit=200)[0]
    assert abs(mass - exact) / exact < 1e-4


def test_single_event_focuses(op_c1):
    """A hyperbolic event with (tau0, q0) on grid nodes focuses there."""
    d = op_c1.desc
    l0, i0 = 70, 180
    tau0 = d.tau0 + i0 * d.dtau
    q0 = d.q0 + l0 * d.dq
    t = np.arange(d.nt) * d.dt
    x = d.x0 + np.arange(d.nx) * d.dx
    te = np.sqrt(tau0 ** 2 + (q0 * x) ** 2)
    f = synth.ricker(t[None, :] - te[:, None], 12.0)
    for g in (op_c1.forward(f), direct.forward(d, f)):
        l, i = np.unravel_index(np.argmax(np.abs(g)), g.shape)
        assert abs(l - l0) <= 1 and abs(i - i0) <= 1


def test_direct_sum_at_zero_slowness_is_the_trapezoid_stack():
    """q = 0, tau on the time grid: the hyperbola is the line t = tau, Keys
    interpolation is exact at nodes, so R f(tau_i, 0) = sum_k w_k f[k][i]."""
    d = ODD.with_(q0=0.0, tau0=0.0, dtau=ODD.dt)
    f, _ = synth.random_pair(d, 5)
    g = direct.forward(d, f)
    w = np.full(d.nx, d.dx)
    w[[0, -1]] *= 0.5
    assert np.abs(g[0] - w @ f[:, :d.ntau]).max() < 1e-13


def test_direct_sum_reproduces_quadratics():
    """Keys' kernel (a = -1/2) reproduces polynomials of degree <= 2, so for
    f = P(t) the sum is sum_k w_k P(t_ik) wherever the taps stay inside."""
    d = ODD
    t = np.arange(d.nt) * d.dt
    P = lambda tt: 0.3 - 1.2 * tt + 2.5 * tt ** 2
    f = np.tile(P(t), (d.nx, 1))
    g = direct.forward(d, f)
    x = d.x0 + np.arange(d.nx) * d.dx
    w = np.full(d.nx, d.dx)
    w[[0, -1]] *= 0.5
    for l in range(0, d.nq, 3):
        for i in range(0, d.ntau, 4):
            q = d.q0 + l * d.dq
            tau = d.tau0 + i * d.dtau
            th = np.sqrt(tau ** 2 + (q * x) ** 2)
            if th.max() / d.dt + 2 < d.nt - 1 and th.min() / d.dt > 1:
                assert abs(g[l, i] - w @ P(th)) < 1e-12


def test_direct_forward_at_matches_vectorised():
    d = ODD
    f, _ = synth.random_pair(d, 9)
    g = direct.forward(d, f)
    for l, i in [(0, 0), (3, 17), (18, 28), (10, 5)]:
        assert abs(direct.forward_at(d, f, l, i) - g[l, i]) < 1e-13


def _periodic(dv, M):
    return dv - M * np.round(dv / M)


def test_brute_force_dense_operator_16x16():
    """Assemble the 16x16 operator twice: (a) by applying the oracle to unit
    vectors, (b) independently, as dense matrices: B-spline smearing over all
    lattice nodes by periodic distance, circulant convolution with the
    kernel's inverse DFT written as an explicit exponential sum, B-spline
    interpolation, scalings.  They agree to 1e-12 and the adjoint's matrix is
    the transpose."""
    d = TINY
    op = logpolar.LogPolarOracle(d)
    g = op.geo
    M1, M2 = g.Mtheta, g.Mrho
    n_in = d.nx * d.nt
    n_out = d.nq * d.ntau
    A = np.zeros((n_out, n_in))
    for c in range(n_in):
        e = np.zeros(n_in)
        e[c] = 1.0
        A[:, c] = op.forward(e.reshape(d.nx, d.nt)).ravel()
    At = np.zeros((n_in, n_out))
    for c in range(n_out):
        e = np.zeros(n_out)
        e[c] = 1.0
        At[:, c] = op.adjoint(e.reshape(d.nq, d.ntau)).ravel()
    assert np.abs(At - A.T).max() < 1e-12 * np.abs(A).max()

    m = np.arange(M1)
    n = np.arange(M2)
    # (b1) smearing matrix, lattice node (m, n) <- data sample (k, j)
    keep = g.keep.ravel()
    xs = (g.phi / g.dtheta).ravel()
    ys = (g.eta / g.drho).ravel()
    Bx = bspline.beta3(_periodic(m[:, None] - xs[None, :], M1))   # (M1, n_in)
    By = bspline.beta3(_periodic(n[:, None] - ys[None, :], M2))   # (M2, n_in)
    S = (Bx[:, None, :] * By[None, :, :]).reshape(M1 * M2, n_in)
    S = S * (g.W.ravel() * keep)[None, :]
    # (b2) kappa = inverse DFT of K by explicit sums, circulant matrix
    k1 = np.arange(M1)
    k2 = np.arange(M2)
    E1 = np.exp(2j * np.pi * np.outer(m, k1) / M1)
    E2 = np.exp(2j * np.pi * np.outer(k2, n) / M2)
    kappa = (E1 @ op.K @ E2).real / (M1 * M2)
    dm = (m[:, None] - m[None, :]) % M1
    dn = (n[:, None] - n[None, :]) % M2
    Cm = kappa[dm[:, None, :, None], dn[None, :, None, :]].reshape(M1 * M2, M1 * M2)
    # (b3) interpolation matrix at the Radon samples, and output scaling
    xo = np.repeat(g.theta / g.dtheta, d.ntau)
    yo = (g.rho / g.drho).ravel()
    Gx = bspline.beta3(_periodic(xo[:, None] - m[None, :], M1))
    Gy = bspline.beta3(_periodic(yo[:, None] - n[None, :], M2))
    G = (Gx[:, :, None] * Gy[:, None, :]).reshape(n_out, M1 * M2)
    G = G * np.repeat(g.out_scale, d.ntau)[:, None]
    B = G @ Cm @ S
    assert np.abs(A - B).max() < 1e-12 * np.abs(A).max()


def test_brute_force_direct_sum_16x16():
    """Dense direct-sum matrix from per-sample evaluation vs the vectorised
    forward, and the adjoint as its transpose."""
    d = TINY
    n_in = d.nx * d.nt
    rng = np.random.default_rng(4)
    f = rng.standard_normal((d.nx, d.nt))
    g = direct.forward(d, f)
    for l in range(0, d.nq, 5):
        for i in range(0, d.ntau, 5):
            assert abs(direct.forward_at(d, f, l, i) - g[l, i]) < 1e-13
    A = np.zeros((d.nq * d.ntau, n_in))
    for c in range(n_in):
        e = np.zeros(n_in)
        e[c] = 1.0
        A[:, c] = direct.forward(d, e.reshape(d.nx, d.nt)).ravel()
    gg = rng.standard_normal((d.nq, d.ntau))
    assert np.abs(direct.adjoint(d, gg).ravel() - A.T @ gg.ravel()).max() < 1e-12
