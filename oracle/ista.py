"""Soft-thresholding iterations and the power iteration for their step size
(oracle, FP64; test infrastructure only).

Section 3 minimises ||R* g - f||^2 + mu ||g||_1 over Radon panels g (eq.
R_ell1) by the iterations of eq. iters,
    g^n = S_{c^2 mu}(g^{n-1} + c^2 R (f - R* g^{n-1})),
with c ||R|| < 1 and the soft threshold
    S_mu(v) = v + mu/2 (v <= -mu/2),  0 (|v| < mu/2),  v - mu/2 (v >= mu/2);
for traces missing outside a recorded set S (eq. itersmd) the residual is
f - chi_S R* g^{n-1}, f being zero where data are missing.

The operators are passed in as callables (the float64 log-polar oracle's
forward and adjoint, or a dense matrix in the tests).  c is fixed from
||R||^2 = largest eigenvalue of R* R, estimated by the power iteration.
"""
from __future__ import annotations

import numpy as np


def soft_threshold(v, mu):
    """S_mu of Section 3 (threshold at mu/2)."""
    v = np.asarray(v, dtype=np.float64)
    h = 0.5 * mu
    return np.where(v >= h, v - h, np.where(v <= -h, v + h, 0.0))


def power_norm2(forward, adjoint, shape, iters=50, seed=0):
    """||R||^2 = max eigenvalue of R* R by the power iteration from a seeded
    uniform start vector: v <- R*R v / |R*R v|, estimate <v, R*R v>, |v| = 1."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.0, 1.0, size=shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = adjoint(forward(v))
        lam = float(np.sum(v * w))
        nw = np.linalg.norm(w)
        if nw == 0.0:
            break
        v = w / nw
    return lam


def objective(forward, adjoint, f, g, mu, mask=None):
    """||chi_S (R* g - f)||^2 + mu ||g||_1 (eqs. R_ell1 and its masked form)."""
    r = adjoint(g) - f
    if mask is not None:
        r = r * mask
    return float(np.sum(r * r) + mu * np.sum(np.abs(g)))


def ista(forward, adjoint, f, iters, c2, mu, mask=None, g0=None):
    """`iters` iterations of eq. itersmd (eq. iters when mask is None)."""
    g = np.zeros_like(forward(np.zeros_like(f))) if g0 is None else np.array(g0, dtype=np.float64)
    for _ in range(iters):
        a = adjoint(g)
        if mask is not None:
            a = a * mask
        g = soft_threshold(g + c2 * forward(f - a), c2 * mu)
    return g
