"""Seeded synthetic inputs shaped like the paper's workloads.

The paper tests on a synthetic CMP gather with N x N samples (Section 5) and on
gathers with randomly missing traces (Section 6.2).  Neither data set ships with
the paper, so these generators stand in for them: sums of hyperbolic events
t = sqrt(tau_e^2 + x^2 / v_e^2) carrying a Ricker wavelet, optional Gaussian
noise and random trace masks.  Everything is drawn from numpy's PCG64 with a
fixed seed; the draw order is tau_e, v_e, A_e, then noise, then mask.

Layouts (the same everywhere in this repository):
  data   f[k][j] = f(t_j, x_k),    t_j = j*dt,            x_k = x0 + k*dx
  Radon  g[l][i] = g(tau_i, q_l),  tau_i = tau0 + i*dtau, q_l = q0 + l*dq
Units: seconds, kilometres, seconds per kilometre.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class GridDesc:
    """Regular sampling of a CMP gather and of its Radon panel."""
    nt: int
    nx: int
    dt: float
    x0: float
    dx: float
    ntau: int
    nq: int
    tau0: float
    dtau: float
    q0: float
    dq: float
    oversample: float = 2.0

    def with_(self, **kw) -> "GridDesc":
        return replace(self, **kw)

    @property
    def T(self) -> float:
        return (self.nt - 1) * self.dt

    @property
    def X(self) -> float:
        return self.x0 + (self.nx - 1) * self.dx


Q_MIN = 1.0 / 4.0      # slowness of v = 4 km/s
Q_MAX = 1.0 / 1.5      # slowness of v = 1.5 km/s


def _desc(nt, dt, nx, xmax, nq=None, ntau=None, sigma=2.0) -> GridDesc:
    nq = nx if nq is None else nq
    ntau = nt if ntau is None else ntau
    return GridDesc(nt=nt, nx=nx, dt=dt, x0=0.0, dx=xmax / (nx - 1),
                    ntau=ntau, nq=nq, tau0=0.0, dtau=dt,
                    q0=Q_MIN, dq=(Q_MAX - Q_MIN) / (nq - 1), oversample=sigma)


# name -> (grid, events, peak frequency Hz, tau range as fraction of T or
#          absolute seconds, noise fraction, seed)
CONFIGS = {
    # single gather, 256 x 128, x in [0, 2] km, 5 events, 25 Hz
    "c1": dict(desc=_desc(256, 0.004, 128, 2.0), events=5, freq=25.0,
               tau=("abs", 0.1, 0.9), noise=0.0, seed=1),
    # single gather, 1024 x 512, x in [0, 4] km, 30 events, 25 Hz, 5 % noise
    "c2": dict(desc=_desc(1024, 0.004, 512, 4.0), events=30, freq=25.0,
               tau=("rel", 0.1, 0.9), noise=0.05, seed=2),
    # large gather, 2048 x 1024, dt = 2 ms, x in [0, 4] km, 100 events, 30 Hz
    "c3": dict(desc=_desc(2048, 0.002, 1024, 4.0), events=100, freq=30.0,
               tau=("rel", 0.1, 0.9), noise=0.0, seed=3),
}


def config_desc(name: str) -> GridDesc:
    return CONFIGS[name]["desc"]


def ricker(t: np.ndarray, freq: float) -> np.ndarray:
    """Ricker wavelet with peak frequency `freq`, r(0) = 1."""
    a = (np.pi * freq * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def ricker_gather(desc: GridDesc, events: int, freq: float, seed: int,
                  tau_range=("rel", 0.1, 0.9), vel=(1.5, 4.0),
                  noise: float = 0.0, dtype=np.float64) -> np.ndarray:
    """Sum of hyperbolic Ricker events, shape (nx, nt)."""
    rng = np.random.default_rng(seed)
    kind, lo, hi = tau_range
    if kind == "rel":
        lo, hi = lo * desc.T, hi * desc.T
    tau_e = rng.uniform(lo, hi, events)
    v_e = rng.uniform(vel[0], vel[1], events)
    amp = rng.normal(0.0, 1.0, events)
    t = np.arange(desc.nt) * desc.dt
    x = desc.x0 + np.arange(desc.nx) * desc.dx
    f = np.zeros((desc.nx, desc.nt))
    for e in range(events):
        te = np.sqrt(tau_e[e] ** 2 + (x / v_e[e]) ** 2)
        f += amp[e] * ricker(t[None, :] - te[:, None], freq)
    if noise > 0.0:
        rms = np.sqrt(np.mean(f * f))
        f += rng.normal(0.0, noise * rms, f.shape)
    return f.astype(dtype)


def s1_desc(n: int) -> GridDesc:
    """Square grids of the size sweep beside the paper's timing tables
    (Nt = Nx = Ntau = Nq = n): t over about 4 s, offsets 0..4 km, slownesses
    for 1.5..4 km/s."""
    return GridDesc(nt=n, nx=n, dt=4.0 / n, x0=0.0, dx=4.0 / (n - 1), ntau=n, nq=n,
                    tau0=0.0, dtau=4.0 / n, q0=Q_MIN, dq=(Q_MAX - Q_MIN) / (n - 1))


def s1_gather(n: int, dtype=np.float64) -> np.ndarray:
    """30 Ricker events of 25 Hz on s1_desc(n) (seed 6)."""
    return ricker_gather(s1_desc(n), 30, 25.0, 6, dtype=dtype)


def config_gather(name: str, dtype=np.float64) -> np.ndarray:
    c = CONFIGS[name]
    return ricker_gather(c["desc"], c["events"], c["freq"], c["seed"],
                         c["tau"], noise=c["noise"], dtype=dtype)


def band_limited_gather(desc: GridDesc, events: int, freq: float, seed: int,
                        tau_range=("rel", 0.7, 0.85), vel=(1.5, 4.0), taper: float = 0.1,
                        dtype=np.float64) -> np.ndarray:
    """Hyperbolic Ricker events (as ricker_gather, no noise) that a single
    log-polar part represents: late events (tau from 0.7 T), a low peak
    frequency chosen by the caller, and a cosine taper to zero over the last
    `taper` fraction of the time axis and of the offsets, so that the record
    has no hard edge at t = T or x = X.  Shape (nx, nt)."""
    f = ricker_gather(desc, events, freq, seed, tau_range, vel)
    t = np.arange(desc.nt) * desc.dt
    x = desc.x0 + np.arange(desc.nx) * desc.dx

    def edge(u, top):
        # 1 below (1 - taper) top, cosine to 0 at top
        r = np.clip((u - (1.0 - taper) * top) / (taper * top), 0.0, 1.0)
        return 0.5 * (1.0 + np.cos(np.pi * r))

    f *= edge(x, desc.X)[:, None] * edge(t, desc.T)[None, :]
    return f.astype(dtype)


def gaussian_sy_gather(desc: GridDesc, cs: float, cy: float, width: float,
                       dtype=np.float64) -> np.ndarray:
    """f(t,x) = 2 xh exp(-((th^2-cs)^2 + (xh^2-cy)^2) / (2 width^2)),
    th = t/T, xh = x/X: an isotropic Gaussian in (s, y) = (th^2, xh^2) once
    divided by 2 sqrt(y).  Shape (nx, nt)."""
    th = np.arange(desc.nt) * desc.dt / desc.T
    xh = (desc.x0 + np.arange(desc.nx) * desc.dx) / desc.X
    s = th[None, :] ** 2
    y = xh[:, None] ** 2
    f = 2.0 * xh[:, None] * np.exp(-((s - cs) ** 2 + (y - cy) ** 2)
                                   / (2.0 * width ** 2))
    return f.astype(dtype)


def trace_mask(nx: int, frac_missing: float, seed: int) -> np.ndarray:
    """Boolean mask over offsets: False for the round(frac*nx) traces drawn
    without replacement."""
    rng = np.random.default_rng(seed)
    miss = rng.choice(nx, int(round(frac_missing * nx)), replace=False)
    m = np.ones(nx, dtype=bool)
    m[miss] = False
    return m


def c5_batch(n: int = 16, frac_missing: float = 0.5):
    """Trace-interpolation workload: n gathers of C2 shape and physics
    (1024 x 512, x in [0, 4] km, 30 events, 25 Hz) without noise, gather b
    drawn with seed 500 + b, and for each a mask over offsets with
    round(frac * 512) traces missing (its own generator, seed 500 + b).
    Returns (desc, [f_b (nx, nt)], [keep_b (nx,) bool])."""
    c = CONFIGS["c2"]
    desc = c["desc"]
    fs, keeps = [], []
    for b in range(n):
        fs.append(ricker_gather(desc, c["events"], c["freq"], 500 + b, c["tau"]))
        keeps.append(trace_mask(desc.nx, frac_missing, 500 + b))
    return desc, fs, keeps


def demultiple_gather(desc: GridDesc, seed: int, primaries: int = 6, multiples: int = 4,
                      freq: float = 25.0, v_prim=(2.2, 4.0), v_mult=(1.5, 1.9)):
    """Primaries (velocities v_prim) plus slower multiples (v_mult, arriving in
    the later 60 % of the record), Ricker events.  Returns (total, primaries,
    multiples), each (nx, nt); with the default velocities every multiple
    has q > 1/1.9 s/km and every primary q < 1/2.2 s/km."""
    prim = ricker_gather(desc, primaries, freq, seed, ("rel", 0.1, 0.9), vel=v_prim)
    mult = ricker_gather(desc, multiples, freq, seed + 1, ("rel", 0.3, 0.9), vel=v_mult)
    return prim + mult, prim, mult


def batch_descs(n: int = 64, seed: int = 4):
    """Uneven batch: nt in {512, 1024, 2048}, nx in {128, ..., 1024} step 128,
    ntau = nt, nq = nx, dt = 2 ms, dx = 4/1023 km."""
    rng = np.random.default_rng(seed)
    nts = rng.choice([512, 1024, 2048], n)
    nxs = rng.choice(np.arange(128, 1025, 128), n)
    dx = 4.0 / 1023.0
    out = []
    for nt, nx in zip(nts, nxs):
        nt, nx = int(nt), int(nx)
        out.append(GridDesc(nt=nt, nx=nx, dt=0.002, x0=0.0, dx=dx,
                            ntau=nt, nq=nx, tau0=0.0, dtau=0.002,
                            q0=Q_MIN, dq=(Q_MAX - Q_MIN) / (nx - 1)))
    return out


def batch_gathers(descs, seed_base: int = 400, dtype=np.float32):
    out = []
    for b, d in enumerate(descs):
        rng = np.random.default_rng(seed_base + b)
        ev = int(rng.integers(10, 61))
        out.append(ricker_gather(d, ev, 30.0, seed_base + b + 10_000,
                                 dtype=dtype))
    return out


def random_pair(desc: GridDesc, seed: int, dtype=np.float64):
    """Standard-normal data panel (nx, nt) and Radon panel (nq, ntau)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((desc.nx, desc.nt))
    g = rng.standard_normal((desc.nq, desc.ntau))
    return f.astype(dtype), g.astype(dtype)
