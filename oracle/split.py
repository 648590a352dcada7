"""Splitting into parts (oracle, FP64; test infrastructure only).

Section 4 (eq. tsplit) cuts the integral over t at an intermediate time, and
may do so repeatedly, so that each piece is evaluated with the log-polar
lattice its own samples call for (eq. lpsamples): the early times, where the
Radon samples crowd together, get a finer lattice.  Section 5 applies one such
cut in time and one in slowness.  The transform of the whole gather is the sum
of the transforms of the pieces.

Readings (the paper gives no more than the cut of the integral):
* S1  A part is (time band [j_lo, j_hi), slowness band [l_lo, l_hi)) and is a
      plain problem of its own, rescaled by its own T and X (eq. hypnorm):
      time samples 0 .. nt_p - 1 with nt_p = min(nt, j_hi + 2), only those
      inside the band taken in (reading R11 of the geometry), and the
      slowness rows of the band (q0_p = q0 + l_lo dq).
* S2  Its Radon samples are those with tau_i <= (nt_p - 1) dt: a data sample
      at t contributes to tau <= t only, and the two extra samples cover the
      reach of the cubic interpolation in time of the direct summation.
* S3  Its traces are those holding a kept sample inside the band,
      (j_hi - 1) dt >= q0_p x_k, plus one, so that the trapezoid-rule
      weight 1/2 of its last trace falls on a trace with nothing kept in the
      band (or on the last trace of the whole grid).
* S4  Time bands cover disjoint data samples; slowness bands disjoint Radon
      rows; the split forward adds the parts' forwards into the whole Radon
      panel and the split adjoint, the parts' adjoints into the whole gather,
      so the split adjoint is the exact transpose of the split forward.
"""
from __future__ import annotations

from dataclasses import dataclass
from types import SimpleNamespace

import numpy as np

from .logpolar import LogPolarOracle

MARGIN = 2  # reading S2
_FIELDS = ("nt", "nx", "dt", "x0", "dx", "ntau", "nq", "tau0", "dtau", "q0", "dq",
           "oversample")


@dataclass
class Part:
    desc: SimpleNamespace
    j_lo: int
    j_hi: int
    l_lo: int
    l_hi: int


def _check_edges(edges, n, what):
    e = [int(v) for v in edges]
    if len(e) < 2 or e[0] != 0 or e[-1] != n or any(b <= a for a, b in zip(e, e[1:])):
        raise ValueError(f"{what} edges must increase from 0 to {n}")
    return e


def parts(desc, t_edges, q_edges) -> list[Part]:
    """The parts of readings S1-S3, part iq * n_t + it for time band it and
    slowness band iq."""
    te = _check_edges(t_edges, desc.nt, "time")
    qe = _check_edges(q_edges, desc.nq, "slowness")
    base = {k: getattr(desc, k) for k in _FIELDS if hasattr(desc, k)}
    base.setdefault("oversample", 2.0)
    x = desc.x0 + np.arange(desc.nx) * desc.dx
    tau = desc.tau0 + np.arange(desc.ntau) * desc.dtau
    out = []
    for iq in range(len(qe) - 1):
        for it in range(len(te) - 1):
            j_lo, j_hi, l_lo, l_hi = te[it], te[it + 1], qe[iq], qe[iq + 1]
            nt_p = min(desc.nt, j_hi + MARGIN)
            q0_p = desc.q0 + l_lo * desc.dq
            n_kept_traces = int(np.count_nonzero((j_hi - 1) * desc.dt >= q0_p * x))
            ntau_p = int(np.count_nonzero(tau <= (nt_p - 1) * desc.dt))
            if n_kept_traces == 0 or ntau_p == 0:
                raise ValueError("a part holds no kept sample or no Radon sample")
            sub = SimpleNamespace(**{**base, "nt": nt_p, "nx": min(desc.nx, n_kept_traces + 1),
                                     "ntau": ntau_p, "nq": l_hi - l_lo, "q0": q0_p})
            out.append(Part(sub, j_lo, j_hi, l_lo, l_hi))
    return out


class SplitOracle:
    """Forward and adjoint of the split transform (reading S4)."""

    def __init__(self, desc, t_edges, q_edges):
        self.desc = desc
        self.parts = parts(desc, t_edges, q_edges)
        self.ops = [LogPolarOracle(p.desc, window=(p.j_lo, p.j_hi)) for p in self.parts]

    def forward(self, f: np.ndarray) -> np.ndarray:
        f = np.asarray(f, dtype=np.float64)
        g = np.zeros((self.desc.nq, self.desc.ntau))
        for p, op in zip(self.parts, self.ops):
            s = p.desc
            g[p.l_lo:p.l_hi, :s.ntau] += op.forward(f[:s.nx, :s.nt])
        return g

    def adjoint(self, g: np.ndarray) -> np.ndarray:
        g = np.asarray(g, dtype=np.float64)
        f = np.zeros((self.desc.nx, self.desc.nt))
        for p, op in zip(self.parts, self.ops):
            s = p.desc
            f[:s.nx, :s.nt] += op.adjoint(g[p.l_lo:p.l_hi, :s.ntau])
        return f
