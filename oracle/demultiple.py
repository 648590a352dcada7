"""Multiple attenuation in the Radon domain (oracle, FP64; test
infrastructure only).

Section 6: primaries and multiples separate in the Radon panel by their
moveout (multiples are slower, so they sit at larger slowness q).  The
sparse panel g of the gather (soft-thresholding iterations, Section 3) is
cut at a border line; the multiples' side is taken back to the gather with
the adjoint and subtracted from it.  Reading: the border is the straight line
q = qb0 + qb_slope tau in the (tau, q) plane, multiples where q > border.
"""
from __future__ import annotations

import numpy as np


def mute_multiples(desc, g, qb0, qb_slope=0.0):
    """g restricted to the multiples' side, q_l > qb0 + qb_slope tau_i."""
    q = desc.q0 + np.arange(desc.nq, dtype=np.float64) * desc.dq
    tau = desc.tau0 + np.arange(desc.ntau, dtype=np.float64) * desc.dtau
    keep = q[:, None] > qb0 + qb_slope * tau[None, :]
    return np.where(keep, g, 0.0)


def demultiple(adjoint, desc, f, g, qb0, qb_slope=0.0):
    """Primaries: f - R* (g on the multiples' side)."""
    return f - adjoint(mute_multiples(desc, g, qb0, qb_slope))
