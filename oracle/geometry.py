"""Geometry of the log-polar set-up (oracle, FP64; test infrastructure only).

Paper passages followed:
* Section 2.2, eq. hypnorm / Qgrid: rescale the gather to the unit square,
  t^ = t/T, x^ = x/X, tau^ = tau/T, q^ = q X/T, result scaled by X.
* Section 2, eqs. f / Rhdef2: s = t^2, y = x^2 turn hyperbolas into lines
  s - q^2 y = tau^2.
* Section 2.1: sector opening beta, mid angle alpha, theta = alpha - arctan q^2,
  the inscribed square of side a at offset O (three corners on the sector
  border), the trapezoid cut t >= k x and the first contribution a_r.
* Section 2.1, eqs. transformT / transformP: T (rotate by alpha, scale by a,
  translate by O) and the polar map P1 (angle, log radius).
* Section 4, eq. lpsamples: lattice spacing from the largest distance between
  neighbouring mapped samples.

Readings (the paper is silent or garbled):
* R1  The transform is one-sided, integral over 0 <= x <= X (data exist for
      x >= 0 only); the two-sided form of eq. Rhdef2 is this times 2.
* R2  O_1 = a sin(alpha + pi/4) / (sqrt(2) tan(beta/2)).  The printed O_1
      (with tan(beta)) does not put corners (0,0) and (1,1) on the sector's
      rays; this value does, and it reproduces the printed a and O_2.
* R3  Corner (s,y) = (0,0) lies on the -beta/2 ray, (1,1) on the +beta/2 ray,
      (1,0) on the unit arc.
* R4  The trapezoid slope is k = q^_min: no hyperbola with q >= q_min
      samples t < q_min x.  A sample is kept iff  j*dt >= q0*(x0 + k*dx)
      evaluated in float64 exactly as written.  a_r = |A| cos(beta), the
      distance of the (tau=0, q_min) line from the origin.
* R5  Radon side: theta_l = alpha - arctan(q^_l^2) and e^rho = distance of
      the mapped line s - q^2 y = tau^2 from the origin
      = A_l + B_l tau^2 (derived directly; the printed map S has a sign
      inconsistency with P2).
* R6  Lattice axis 0 is the angle (k1), axis 1 the log radius (k2).
* R7  Output factor X cos(psi_l)/a with psi_l = arctan(q^_l^2): the
      delta-function rescaling of the rotated, dilated set-up.
* R8  Smear weight W = 2 a^2 t^ e^-eta w_t w_x dt^ dx^ (trapezoid rule in t
      and x; the 1/(2x) of eq. f cancels against the Jacobian, eq. B3tx).
* R9  Spacing: dtheta0, drho0 are the literal maxima of eq. lpsamples over
      neighbour pairs with both samples kept; the lattice uses
      dtheta = dtheta0/sigma, drho = drho0/sigma, sigma the oversampling.
* R11 A part of a split (Section 4, eq. tsplit) takes in only the data
      samples of its time band [j_lo, j_hi): the kept set is the trapezoid
      intersected with the band, everywhere above (maxima of eq. lpsamples,
      smear weights, kept points).
* R10 Extent: beta_k = beta + 4 dtheta; M_theta = smallest even 5-smooth
      integer >= ceil(2 beta_k/dtheta) + 1; M_rho = smallest even 5-smooth
      integer >= ceil((|ln a_r| + |ln cos beta_k|)/drho) + 9.  Node m sits at
      theta = m dtheta, node n at rho = n drho, indices taken mod M.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def next_even_smooth(n: int) -> int:
    """Smallest even integer >= n whose prime factors are 2, 3, 5 only."""
    m = max(int(n), 2)
    while True:
        if m % 2 == 0:
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                return m
        m += 1


@dataclass
class Geometry:
    # rescaling (eq. hypnorm)
    T: float
    X: float
    that: np.ndarray     # (nt,)
    xhat: np.ndarray     # (nx,)
    tauhat: np.ndarray   # (ntau,)
    qhat: np.ndarray     # (nq,)
    # sector and square (Section 2.1)
    alpha: float
    beta: float
    a: float
    O1: float
    O2: float
    a_r: float
    kslope: float
    # data side, shape (nx, nt)
    keep: np.ndarray
    phi: np.ndarray      # angle of the mapped sample
    eta: np.ndarray      # log radius of the mapped sample
    W: np.ndarray        # smear weight, 0 where not kept
    # Radon side
    psi: np.ndarray      # (nq,) arctan(q^2)
    theta: np.ndarray    # (nq,) alpha - psi
    rho: np.ndarray      # (nq, ntau)
    out_scale: np.ndarray  # (nq,) X cos(psi)/a
    # lattice
    sigma: float
    dtheta0: float
    drho0: float
    dtheta: float
    drho: float
    beta_k: float
    Mtheta: int
    Mrho: int

    @property
    def Ptheta(self) -> float:
        return self.Mtheta * self.dtheta

    @property
    def Prho(self) -> float:
        return self.Mrho * self.drho


def sector(qh_min: float, qh_max: float):
    """alpha, beta, a, O1, O2, a_r for rescaled slownesses (Section 2.1;
    readings R2-R4)."""
    psi_min = math.atan(qh_min * qh_min)
    psi_max = math.atan(qh_max * qh_max)
    beta = psi_max - psi_min
    alpha = 0.5 * (psi_max + psi_min)
    s2a = math.sin(2.0 * alpha)
    a = math.sin(beta) / math.sqrt(s2a * math.sin(beta)
                                   + math.cos(beta) * (s2a + math.sin(beta))
                                   + 1.0)
    O1 = a * math.sin(alpha + math.pi / 4) / (math.sqrt(2.0) * math.tan(beta / 2))
    O2 = a * math.cos(alpha + math.pi / 4) * math.tan(beta / 2) / math.sqrt(2.0)
    # corner A = T(0, 0)
    Au, Av = map_T(0.0, 0.0, alpha, a, O1, O2)
    a_r = math.hypot(Au, Av) * math.cos(beta)
    return alpha, beta, a, O1, O2, a_r


def map_T(s, y, alpha, a, O1, O2):
    """Affine map T of eq. transformT applied to (s, y) = (t^2, x^2)."""
    ds = np.asarray(s) - 0.5
    dy = np.asarray(y) - 0.5
    u = a * (math.cos(alpha) * ds - math.sin(alpha) * dy) + O1
    v = a * (math.sin(alpha) * ds + math.cos(alpha) * dy) + O2
    return u, v


def map_P1(u, v):
    """Polar map of eq. transformP: (angle, log radius) of the point (u, v)."""
    return np.arctan2(v, u), 0.5 * np.log(u * u + v * v)


def kept_mask(desc) -> np.ndarray:
    """Trapezoid of reading R4: keep (j, k) iff j*dt >= q0*(x0 + k*dx)."""
    j = np.arange(desc.nt, dtype=np.float64)
    k = np.arange(desc.nx, dtype=np.float64)
    t = j * desc.dt
    x = desc.x0 + k * desc.dx
    return t[None, :] >= desc.q0 * x[:, None]


def trapezoid_weights(n: int) -> np.ndarray:
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def validate(desc) -> None:
    if min(desc.nt, desc.nx, desc.ntau, desc.nq) < 4:
        raise ValueError("every grid needs at least 4 samples")
    if min(desc.dt, desc.dx, desc.dtau, desc.dq) <= 0.0:
        raise ValueError("sampling intervals must be positive")
    if desc.q0 < 0.0 or desc.x0 < 0.0 or desc.tau0 < 0.0:
        raise ValueError("need q0 >= 0, x0 >= 0, tau0 >= 0")
    if desc.tau0 + (desc.ntau - 1) * desc.dtau > (desc.nt - 1) * desc.dt:
        raise ValueError("tau range exceeds the time range")
    if desc.oversample < 1.5:
        raise ValueError("oversampling must be >= 1.5")


def build(desc, window=None) -> Geometry:
    """Everything of Sections 2.1, 2.2 and 4 that depends only on the grids;
    `window` = (j_lo, j_hi) restricts the kept data samples to a time band
    (reading R11)."""
    validate(desc)
    T = (desc.nt - 1) * desc.dt
    X = desc.x0 + (desc.nx - 1) * desc.dx
    t = np.arange(desc.nt) * desc.dt
    x = desc.x0 + np.arange(desc.nx) * desc.dx
    tau = desc.tau0 + np.arange(desc.ntau) * desc.dtau
    q = desc.q0 + np.arange(desc.nq) * desc.dq
    that, xhat, tauhat, qhat = t / T, x / X, tau / T, q * X / T

    alpha, beta, a, O1, O2, a_r = sector(qhat[0], qhat[-1])

    # data samples: (s, y) = (t^2, x^2) -> T -> P1
    s = that[None, :] ** 2 * np.ones((desc.nx, 1))
    y = xhat[:, None] ** 2 * np.ones((1, desc.nt))
    u, v = map_T(s, y, alpha, a, O1, O2)
    phi, eta = map_P1(u, v)
    keep = kept_mask(desc)
    if window is not None:
        j = np.arange(desc.nt)
        keep = keep & ((j >= window[0]) & (j < window[1]))[None, :]

    # smear weight, reading R8
    dth = desc.dt / T
    dxh = desc.dx / X
    W = (2.0 * a * a * that[None, :] * np.exp(-eta)
         * trapezoid_weights(desc.nt)[None, :]
         * trapezoid_weights(desc.nx)[:, None] * dth * dxh)
    W = np.where(keep, W, 0.0)

    # Radon samples, reading R5
    psi = np.arctan(qhat ** 2)
    theta = alpha - psi
    A_l = (O1 * np.cos(theta) + O2 * np.sin(theta)
           + 0.5 * a * (np.sin(psi) - np.cos(psi)))
    B_l = a * np.cos(psi)
    rho = np.log(A_l[:, None] + B_l[:, None] * tauhat[None, :] ** 2)
    out_scale = X * np.cos(psi) / a

    # lattice spacing, eq. lpsamples with reading R9
    both_t = keep[:, 1:] & keep[:, :-1]
    both_x = keep[1:, :] & keep[:-1, :]
    dth0 = max(np.abs(np.diff(phi, axis=1))[both_t].max(),
               np.abs(np.diff(phi, axis=0))[both_x].max())
    drh0 = max(np.abs(np.diff(eta, axis=1))[both_t].max(),
               np.abs(np.diff(eta, axis=0))[both_x].max())
    sigma = float(desc.oversample)
    dtheta = dth0 / sigma
    drho = drh0 / sigma
    beta_k = beta + 4.0 * dtheta
    Mtheta = next_even_smooth(math.ceil(2.0 * beta_k / dtheta) + 1)
    Mrho = next_even_smooth(
        math.ceil((abs(math.log(a_r)) + abs(math.log(math.cos(beta_k)))) / drho)
        + 9)

    return Geometry(T=T, X=X, that=that, xhat=xhat, tauhat=tauhat, qhat=qhat,
                    alpha=alpha, beta=beta, a=a, O1=O1, O2=O2, a_r=a_r,
                    kslope=qhat[0], keep=keep, phi=phi, eta=eta, W=W,
                    psi=psi, theta=theta, rho=rho, out_scale=out_scale,
                    sigma=sigma, dtheta0=dth0, drho0=drh0, dtheta=dtheta,
                    drho=drho, beta_k=beta_k, Mtheta=Mtheta, Mrho=Mrho)
