"""Spectrum of the log-polar kernel (oracle, FP64; test infrastructure only).

Section 2.1, eqs. lpfwd / finiteconv: the log-polar Radon transform is a
convolution with zeta(theta, rho) = delta(cos theta - e^rho), whose Fourier
transform is evaluated numerically in a precomputing step.  Section 2.2, eqs.
d / lok / B3tauq: the lattice spectrum is multiplied by the kernel spectrum,
divided by the B-spline transform (once for the smearing, once for the final
interpolation) and restricted to the rectangle L.

Readings:
* K1  zeta(theta, rho) = delta(rho - ln cos theta) / cos theta, truncated to
      |theta| <= beta_k (beta_k = beta + 4 dtheta: output and input angles each
      span beta, widened by two lattice cells of spline support per side), so
      zeta^(xi1, xi2) = int_{-beta_k}^{beta_k} sec(theta)
                          exp(-2 pi i (xi1 theta + xi2 ln cos theta)) dtheta,
      evaluated here by composite Gauss-Legendre quadrature.
* K2  On the lattice, frequencies are xi1 = k1/P_theta, xi2 = k2/P_rho with
      signed k in [-M/2, M/2).
* K3  L = { 2 sigma |k1| < M_theta  and  2 sigma |k2| < M_rho } (strict, so the
      Nyquist bins are excluded and K stays Hermitian).
* K4  K[k] = chi_L zeta^(k) / (dtheta drho b(k1/M_theta)^2 b(k2/M_rho)^2),
      b = Fourier transform of B_3 (the 1/(dtheta drho) turns lattice sums into
      integrals).
"""
from __future__ import annotations

import math

import numpy as np

from .bspline import beta3_ft


def signed_freqs(M: int) -> np.ndarray:
    """Signed DFT indices in FFT order: 0, 1, ..., M/2-1, -M/2, ..., -1."""
    return np.fft.fftfreq(M, d=1.0 / M).astype(np.int64)


def in_band(k, M: int, sigma: float) -> np.ndarray:
    """chi_L along one axis (reading K3)."""
    return 2.0 * sigma * np.abs(np.asarray(k, dtype=np.float64)) < M


def quadrature(beta_k: float, n_panels: int, order: int = 20):
    """Composite Gauss-Legendre nodes and weights on [-beta_k, beta_k]."""
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(-beta_k, beta_k, n_panels + 1)
    half = 0.5 * np.diff(edges)
    mid = 0.5 * (edges[1:] + edges[:-1])
    nodes = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    weights = (half[:, None] * w[None, :]).ravel()
    return nodes, weights


def default_panels(geo) -> int:
    """Enough panels for about one oscillation of the phase per panel."""
    k1max = geo.Mtheta / (2.0 * geo.sigma)
    k2max = geo.Mrho / (2.0 * geo.sigma)
    rate = k1max / geo.Ptheta + k2max * math.tan(geo.beta_k) / geo.Prho
    return int(math.ceil(2.0 * geo.beta_k * rate)) + 4


def zeta_hat(geo, k1, k2, n_panels: int | None = None, order: int = 20,
             chunk: int = 4096) -> np.ndarray:
    """zeta^(k1/P_theta, k2/P_rho) for integer arrays k1, k2 (reading K1).

    The integrand separates in k1 and k2, so the quadrature sum is the matrix
    product E1 @ E2 with E1[k1, n] = exp(-2 pi i k1 theta_n / P_theta) and
    E2[n, k2] = w_n sec(theta_n) exp(-2 pi i k2 ln cos(theta_n) / P_rho)."""
    if n_panels is None:
        n_panels = default_panels(geo)
    nodes, weights = quadrature(geo.beta_k, n_panels, order)
    k1 = np.asarray(k1, dtype=np.float64)
    k2 = np.asarray(k2, dtype=np.float64)
    out = np.zeros((k1.size, k2.size), dtype=np.complex128)
    for c0 in range(0, nodes.size, chunk):
        th = nodes[c0:c0 + chunk]
        wt = weights[c0:c0 + chunk]
        E1 = np.exp(-2j * np.pi * np.outer(k1, th) / geo.Ptheta)
        lc = np.log(np.cos(th))
        E2 = (wt / np.cos(th))[:, None] * np.exp(
            -2j * np.pi * np.outer(lc, k2) / geo.Prho)
        out += E1 @ E2
    return out


def kernel_full(geo, n_panels: int | None = None) -> np.ndarray:
    """The lattice multiplier K of reading K4 as an (M_theta, M_rho) complex
    array in FFT order (zero outside L)."""
    k1 = signed_freqs(geo.Mtheta)
    k2 = signed_freqs(geo.Mrho)
    b1 = in_band(k1, geo.Mtheta, geo.sigma)
    b2 = in_band(k2, geo.Mrho, geo.sigma)
    zh = zeta_hat(geo, k1[b1], k2[b2], n_panels)
    den = (geo.dtheta * geo.drho
           * beta3_ft(k1[b1] / geo.Mtheta)[:, None] ** 2
           * beta3_ft(k2[b2] / geo.Mrho)[None, :] ** 2)
    K = np.zeros((geo.Mtheta, geo.Mrho), dtype=np.complex128)
    K[np.ix_(b1, b2)] = zh / den
    return K
