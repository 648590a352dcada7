"""Pins of the multiple-attenuation oracle (Section 6): the mute's border
rule, the two limiting borders, and on seeded primaries + multiples the
output moving toward the true primaries."""
import numpy as np
import pytest

import synth
from oracle import demultiple, ista, logpolar

C1 = synth.config_desc("c1")


def test_mute_limits_and_border_monotonicity():
    g = np.random.default_rng(1).standard_normal((C1.nq, C1.ntau))
    q_hi = C1.q0 + (C1.nq - 1) * C1.dq
    assert not demultiple.mute_multiples(C1, g, q_hi + 1e-9).any()
    np.testing.assert_array_equal(demultiple.mute_multiples(C1, g, C1.q0 - 1e-9), g)
    # a rising border keeps fewer slownesses at later tau, always an upper range
    m = demultiple.mute_multiples(C1, np.ones_like(g), 0.4, 0.1) != 0
    counts = m.sum(axis=0)
    assert np.all(np.diff(counts) <= 0) and counts[0] > counts[-1]
    for i in range(C1.ntau):
        col = m[:, i]
        if col.any():
            first = np.argmax(col)
            assert col[first:].all() and not col[:first].any()


def test_limiting_borders_give_f_and_f_minus_adjoint():
    ora = logpolar.LogPolarOracle(C1)
    f, g = synth.random_pair(C1, 2)
    q_hi = C1.q0 + (C1.nq - 1) * C1.dq
    np.testing.assert_array_equal(demultiple.demultiple(ora.adjoint, C1, f, g, q_hi + 1.0), f)
    np.testing.assert_allclose(demultiple.demultiple(ora.adjoint, C1, f, g, C1.q0 - 1.0),
                               f - ora.adjoint(g), rtol=0, atol=1e-12)


def test_attenuates_synthetic_multiples():
    """30 soft-thresholding iterations, border at q = 1/2.05 s/km between the
    primaries (v >= 2.2 km/s) and the multiples (v <= 1.9 km/s): the output is
    closer to the true primaries than the input by a clear margin."""
    ora = logpolar.LogPolarOracle(C1)
    f, prim, mult = synth.demultiple_gather(C1, 21)
    lam = ista.power_norm2(ora.forward, ora.adjoint, (C1.nx, C1.nt), iters=30, seed=0)
    mu = 0.01 * np.abs(ora.forward(f)).max()
    g = ista.ista(ora.forward, ora.adjoint, f, 30, 0.99 / lam, mu)
    out = demultiple.demultiple(ora.adjoint, C1, f, g, 1 / 2.05)
    before = np.linalg.norm(f - prim)
    after = np.linalg.norm(out - prim)
    assert after <= 0.6 * before
