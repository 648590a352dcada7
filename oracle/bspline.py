"""Cubic cardinal B-spline (oracle, FP64; test infrastructure only).

Section 2.2 resamples between the (t, x), log-polar and (tau, q) domains with
the cubic cardinal B-spline B_3 and compensates for its smoothing by dividing
by its Fourier transform on the rectangle L (eq. d, eq. B3tauq).

Reading: B_3 is the centred cardinal cubic B-spline on [-2, 2] (unit integral,
partition of unity), and its Fourier transform, with the e^{-2 pi i xi x}
convention, is the closed form (sin(pi xi)/(pi xi))^4.
"""
from __future__ import annotations

import numpy as np


def beta3(x):
    """B_3(x): 2/3 - x^2 + |x|^3/2 on |x| <= 1, (2-|x|)^3/6 on 1 <= |x| <= 2,
    zero elsewhere."""
    ax = np.abs(np.asarray(x, dtype=np.float64))
    inner = 2.0 / 3.0 - ax * ax + 0.5 * ax ** 3
    outer = (2.0 - ax) ** 3 / 6.0
    return np.where(ax <= 1.0, inner, np.where(ax < 2.0, outer, 0.0))


def beta3_ft(xi):
    """Fourier transform of B_3 at frequency xi (cycles per unit)."""
    return np.sinc(np.asarray(xi, dtype=np.float64)) ** 4


def taps(coord):
    """Lattice taps of a point at fractional lattice coordinate `coord`.

    Returns (first index, 4 weights): the point touches nodes
    i0-1, i0, i0+1, i0+2 with i0 = floor(coord), node n getting
    B_3(n - coord)."""
    c = np.asarray(coord, dtype=np.float64)
    i0 = np.floor(c).astype(np.int64)
    w = np.stack([beta3((i0 + d) - c) for d in (-1, 0, 1, 2)], axis=-1)
    return i0 - 1, w
