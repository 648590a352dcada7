"""Plain FP64 log-polar hyperbolic Radon transform and its transpose (oracle;
test infrastructure only).

This is the discrete operator of Sections 2.1-2.2 written out step by step, in
the paper's order, with no blocking, pruning or fusion:

forward (Section 2.2, eqs. f, transformT, transformP, B3tx2, lok, B3tauq):
  1. each kept data sample (t_j, x_k) is mapped by (t^2, x^2) -> T -> P1 to
     log-polar coordinates (phi_jk, eta_jk) and smeared onto the equally
     spaced (theta, rho) lattice with the cubic B-spline, carrying weight
     W_jk f_jk (the 1/(2 sqrt y) factor of eq. f times the Jacobian and the
     trapezoid rule, eq. B3tx2);
  2. 2-D DFT of the lattice, multiplication by the kernel multiplier K
     (kernel spectrum / B-spline transforms, restricted to L), inverse DFT;
  3. cubic B-spline interpolation of the result at the log-polar position
     (theta_l, rho_il) of every Radon sample, times X cos(psi_l)/a.
adjoint (Section 3, eq. inner: the exact transpose, by reversing the order):
  spread the Radon samples with weights X cos(psi_l)/a, multiply by conj(K),
  interpolate at the data samples and multiply by W_jk.

Lattice indices are taken modulo the lattice size (circular convolution), node
(m, n) sitting at (m dtheta, n drho).
"""
from __future__ import annotations

import numpy as np

from . import geometry, kernel
from .bspline import taps


def spread(xc, yc, w, M1: int, M2: int) -> np.ndarray:
    """H[m, n] = sum_p w_p B3(m - xc_p) B3(n - yc_p), indices mod (M1, M2)."""
    i1, w1 = taps(xc)
    i2, w2 = taps(yc)
    idx = []
    val = []
    for a in range(4):
        for b in range(4):
            idx.append(((i1 + a) % M1) * M2 + (i2 + b) % M2)
            val.append(w * w1[:, a] * w2[:, b])
    H = np.bincount(np.concatenate(idx), weights=np.concatenate(val),
                    minlength=M1 * M2)
    return H.reshape(M1, M2)


def gather(C: np.ndarray, xc, yc) -> np.ndarray:
    """sum_{m,n} C[m, n] B3(xc - m) B3(yc - n) at every point (xc, yc)."""
    M1, M2 = C.shape
    i1, w1 = taps(xc)
    i2, w2 = taps(yc)
    out = np.zeros(np.shape(xc))
    for a in range(4):
        for b in range(4):
            out += C[(i1 + a) % M1, (i2 + b) % M2] * w1[:, a] * w2[:, b]
    return out


def convolve(H: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Re IDFT2(DFT2(H) * K); the imaginary part vanishes because K is
    Hermitian (checked)."""
    C = np.fft.ifft2(np.fft.fft2(H) * K)
    scale = max(np.abs(C.real).max(), 1e-300)
    if np.abs(C.imag).max() > 1e-9 * scale:
        raise AssertionError("lattice convolution is not real: K not Hermitian")
    return C.real


class LogPolarOracle:
    """Plan (geometry, kernel multiplier, point coordinates) plus forward and
    adjoint of the plain method for one grid description."""

    def __init__(self, desc, n_panels: int | None = None, window=None):
        self.desc = desc
        g = self.geo = geometry.build(desc, window)
        self.K = kernel.kernel_full(g, n_panels)
        # data points inside the trapezoid, in lattice units
        self.kept = np.nonzero(g.keep)
        self.d_x = g.phi[self.kept] / g.dtheta
        self.d_y = g.eta[self.kept] / g.drho
        self.d_w = g.W[self.kept]
        # Radon points in lattice units
        self.r_x = np.broadcast_to(g.theta[:, None] / g.dtheta, g.rho.shape).ravel()
        self.r_y = (g.rho / g.drho).ravel()
        self.r_w = np.broadcast_to(g.out_scale[:, None], g.rho.shape).ravel()

    @property
    def lattice_shape(self):
        return self.geo.Mtheta, self.geo.Mrho

    def forward(self, f: np.ndarray) -> np.ndarray:
        """g = R_h f, f of shape (nx, nt), g of shape (nq, ntau)."""
        f = np.asarray(f, dtype=np.float64)
        M1, M2 = self.lattice_shape
        H = spread(self.d_x, self.d_y, self.d_w * f[self.kept], M1, M2)
        C = convolve(H, self.K)
        F = gather(C, self.r_x, self.r_y)
        return (self.r_w * F).reshape(self.desc.nq, self.desc.ntau)

    def adjoint(self, g: np.ndarray) -> np.ndarray:
        """f* = R_h^T g, g of shape (nq, ntau), f* of shape (nx, nt)."""
        g = np.asarray(g, dtype=np.float64)
        M1, M2 = self.lattice_shape
        H = spread(self.r_x, self.r_y, self.r_w * g.ravel(), M1, M2)
        C = convolve(H, np.conj(self.K))
        out = np.zeros((self.desc.nx, self.desc.nt))
        out[self.kept] = self.d_w * gather(C, self.d_x, self.d_y)
        return out
