"""Direct summation over hyperbolas and its transpose (oracle, FP64; test
infrastructure only).

Eq. (1) (label Rhdef) defines R_h f(tau, q) as the integral of f along the
hyperbola t = sqrt(tau^2 + q^2 x^2).  Section 5 uses its direct evaluation,
with cubic interpolation in time, as the reference method.

Readings:
* D1  One-sided integral over the measured offsets 0 <= x <= X (the data are
      zero elsewhere, eq. Rgrid), by the trapezoid rule in x:
      weights dx/2 at the first and last trace, dx elsewhere.
* D2  "Cubic interpolation" in time is Keys' cubic convolution with
      a = -1/2; samples outside 0 <= j < nt are zero.
* D3  The adjoint is the exact transpose of the discrete sum.
"""
from __future__ import annotations

import numpy as np

KEYS_A = -0.5


def keys(s):
    """Keys cubic convolution kernel with a = -1/2."""
    a = KEYS_A
    x = np.abs(np.asarray(s, dtype=np.float64))
    near = (a + 2.0) * x ** 3 - (a + 3.0) * x ** 2 + 1.0
    far = a * x ** 3 - 5.0 * a * x ** 2 + 8.0 * a * x - 4.0 * a
    return np.where(x <= 1.0, near, np.where(x < 2.0, far, 0.0))


def _grids(desc):
    t_x = desc.x0 + np.arange(desc.nx) * desc.dx
    tau = desc.tau0 + np.arange(desc.ntau) * desc.dtau
    q = desc.q0 + np.arange(desc.nq) * desc.dq
    wx = np.full(desc.nx, desc.dx)
    wx[0] *= 0.5
    wx[-1] *= 0.5
    return t_x, tau, q, wx


def _taps(desc, tau, q_l, x):
    """Time-sample taps of the hyperbola through every (tau_i, x_k) at q_l."""
    t = np.sqrt(tau[:, None] ** 2 + (q_l * x[None, :]) ** 2)
    c = t / desc.dt
    j0 = np.floor(c).astype(np.int64)
    out = []
    for d in (-1, 0, 1, 2):
        m = j0 + d
        w = keys(c - m)
        ok = (m >= 0) & (m < desc.nt)
        out.append((np.where(ok, m, 0), np.where(ok, w, 0.0)))
    return out


def forward(desc, f: np.ndarray, rows=None) -> np.ndarray:
    """g[l][i] = sum_k w_k sum_m f[k][m] keys(t_ilk/dt - m).  `rows` selects
    a subset of slowness indices l (default: all)."""
    f = np.asarray(f, dtype=np.float64)
    x, tau, q, wx = _grids(desc)
    rows = range(desc.nq) if rows is None else rows
    kk = np.arange(desc.nx)[None, :]
    out = []
    for l in rows:
        acc = np.zeros((desc.ntau, desc.nx))
        for m, w in _taps(desc, tau, q[l], x):
            acc += w * f[kk, m]
        out.append(acc @ wx)
    return np.array(out)


def forward_at(desc, f: np.ndarray, l: int, i: int) -> float:
    """One output sample g[l][i], summed trace by trace."""
    f = np.asarray(f, dtype=np.float64)
    x, tau, q, wx = _grids(desc)
    total = 0.0
    for k in range(desc.nx):
        t = np.sqrt(tau[i] ** 2 + (q[l] * x[k]) ** 2)
        c = t / desc.dt
        j0 = int(np.floor(c))
        acc = 0.0
        for m in range(j0 - 1, j0 + 3):
            if 0 <= m < desc.nt:
                acc += f[k, m] * float(keys(c - m))
        total += wx[k] * acc
    return total


def adjoint(desc, g: np.ndarray) -> np.ndarray:
    """f*[k][m] = sum_{l,i} g[l][i] w_k keys(t_ilk/dt - m)."""
    g = np.asarray(g, dtype=np.float64)
    x, tau, q, wx = _grids(desc)
    kk = np.broadcast_to(np.arange(desc.nx)[None, :], (desc.ntau, desc.nx))
    out = np.zeros(desc.nx * desc.nt)
    for l in range(desc.nq):
        gl = g[l][:, None] * wx[None, :]
        for m, w in _taps(desc, tau, q[l], x):
            out += np.bincount((kk * desc.nt + m).ravel(),
                               weights=(gl * w).ravel(),
                               minlength=desc.nx * desc.nt)
    return out.reshape(desc.nx, desc.nt)
