"""Pins for the B-spline and the kernel spectrum (Section 2.1 eq. finiteconv,
Section 2.2 eqs. d, B3tauq)."""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import bspline, geometry, kernel


def test_beta3_partition_of_unity_and_first_moment():
    x = np.linspace(-3.0, 3.0, 1001)
    m = np.arange(-6, 7)
    vals = bspline.beta3(x[:, None] - m[None, :])
    assert np.abs(vals.sum(axis=1) - 1.0).max() < 1e-15
    assert np.abs((vals * m[None, :]).sum(axis=1) - x).max() < 1e-14


def test_beta3_support_and_values():
    assert bspline.beta3(0.0) == pytest.approx(2.0 / 3.0, abs=1e-16)
    assert bspline.beta3(1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert bspline.beta3(2.0) == 0.0 and bspline.beta3(-2.5) == 0.0
    # value and slope are continuous at the knots: the second difference
    # across a knot is O(e^2)
    for k in (1.0, 2.0):
        e = 1e-6
        d2 = bspline.beta3(k - e) + bspline.beta3(k + e) - 2 * bspline.beta3(k)
        assert abs(d2) < 1e-11


def test_beta3_fourier_transform_is_sinc4():
    """B_3 = box * box * box * box, so its transform is sinc^4; check by
    direct quadrature of the piecewise polynomial."""
    for xi in [0.0, 0.05, 0.125, 0.25, 0.4, 0.75]:
        re = integrate.quad(lambda x: float(bspline.beta3(x)) * math.cos(2 * math.pi * xi * x),
                            -2, 2, points=[-1, 0, 1], epsabs=1e-15, epsrel=1e-14)[0]
        assert abs(re - float(bspline.beta3_ft(xi))) < 1e-13


def test_taps_match_definition():
    rng = np.random.default_rng(3)
    c = rng.uniform(-20, 20, 200)
    i0, w = bspline.taps(c)
    for p in range(c.size):
        for d in range(4):
            assert w[p, d] == pytest.approx(float(bspline.beta3(i0[p] + d - c[p])), abs=1e-16)
        assert abs(w[p].sum() - 1) < 1e-15


@pytest.fixture(scope="module")
def geo_c1():
    return geometry.build(synth.config_desc("c1"))


def test_zeta_hat_at_zero_frequency(geo_c1):
    """zeta^(0,0) = int sec = 2 ln(sec beta_k + tan beta_k)."""
    g = geo_c1
    z = kernel.zeta_hat(g, [0], [0])[0, 0]
    exact = 2 * math.log(1 / math.cos(g.beta_k) + math.tan(g.beta_k))
    assert abs(z - exact) < 1e-13 * exact


def test_zeta_hat_against_adaptive_quadrature(geo_c1):
    """Independent evaluation of the kernel-spectrum integral (reading K1) by
    adaptive quadrature of its real and imaginary parts."""
    g = geo_c1
    ks = [(0, 5), (7, 0), (13, -21), (-40, 60), (60, 45)]
    z = kernel.zeta_hat(g, [k[0] for k in ks], [k[1] for k in ks])
    for n, (k1, k2) in enumerate(ks):
        def ph(th):
            return 2 * math.pi * (k1 * th / g.Ptheta + k2 * math.log(math.cos(th)) / g.Prho)
        re = integrate.quad(lambda th: math.cos(ph(th)) / math.cos(th), -g.beta_k, g.beta_k,
                            limit=400, epsabs=1e-14, epsrel=1e-13)[0]
        im = integrate.quad(lambda th: -math.sin(ph(th)) / math.cos(th), -g.beta_k, g.beta_k,
                            limit=400, epsabs=1e-14, epsrel=1e-13)[0]
        assert abs(z[n, n] - complex(re, im)) < 1e-11


def test_zeta_hat_symmetries_and_convergence(geo_c1):
    g = geo_c1
    k1 = kernel.signed_freqs(g.Mtheta)
    k2 = kernel.signed_freqs(g.Mrho)
    k1 = k1[kernel.in_band(k1, g.Mtheta, g.sigma)]
    k2 = k2[kernel.in_band(k2, g.Mrho, g.sigma)]
    z = kernel.zeta_hat(g, k1, k2)
    zneg1 = kernel.zeta_hat(g, -k1, k2)
    zneg = kernel.zeta_hat(g, -k1, -k2)
    scale = np.abs(z).max()
    assert np.abs(z - zneg1).max() < 1e-13 * scale          # even in theta
    assert np.abs(zneg - np.conj(z)).max() < 1e-13 * scale  # real kernel
    p = kernel.default_panels(g)
    z2 = kernel.zeta_hat(g, k1, k2, n_panels=2 * p)
    assert np.abs(z2 - z).max() < 1e-13 * scale


def test_kernel_multiplier_is_hermitian_and_band_limited(geo_c1):
    g = geo_c1
    K = kernel.kernel_full(g)
    # K[-k] = conj K[k]
    Kneg = np.roll(np.flip(K, axis=(0, 1)), shift=(1, 1), axis=(0, 1))
    assert np.abs(Kneg - np.conj(K)).max() < 1e-12 * np.abs(K).max()
    k1 = kernel.signed_freqs(g.Mtheta)
    k2 = kernel.signed_freqs(g.Mrho)
    outside = ~(kernel.in_band(k1, g.Mtheta, g.sigma)[:, None]
                & kernel.in_band(k2, g.Mrho, g.sigma)[None, :])
    assert np.all(K[outside] == 0)
    # at sigma = 2, exactly a quarter band on each axis survives
    assert kernel.in_band(k1, g.Mtheta, 2.0).sum() == 2 * math.ceil(g.Mtheta / 4) - 1
    # value check at the origin: zeta^(0,0)/(dtheta drho)
    z00 = 2 * math.log(1 / math.cos(g.beta_k) + math.tan(g.beta_k))
    assert abs(K[0, 0] - z00 / (g.dtheta * g.drho)) < 1e-12 * abs(K[0, 0])
