"""Pins of the soft-thresholding oracle (Section 3, eqs. iters, itersmd):
the threshold's closed form, the power iteration against a dense
eigensolver, monotone decrease of the objective, and the optimality
conditions of the minimisation at the converged point."""
import numpy as np
import pytest

import synth
from oracle import ista, logpolar

TINY = synth.GridDesc(nt=16, nx=16, dt=0.01, x0=0.0, dx=0.02, ntau=16, nq=16,
                      tau0=0.0, dtau=0.01, q0=0.25, dq=(1 / 1.5 - 0.25) / 15)


def data_mask(desc, frac, seed):
    """chi_S over the (x, t) grid: whole traces missing."""
    keep = synth.trace_mask(desc.nx, frac, seed)
    return np.repeat(keep[:, None], desc.nt, axis=1).astype(np.float64)


@pytest.fixture(scope="module")
def dense():
    """The float64 log-polar operator on 16 x 16 grids as a dense matrix
    (columns = images of the unit vectors)."""
    ora = logpolar.LogPolarOracle(TINY)
    n = TINY.nx * TINY.nt
    A = np.empty((TINY.nq * TINY.ntau, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = ora.forward(e.reshape(TINY.nx, TINY.nt)).ravel()
    fwd = lambda f: (A @ np.ravel(f)).reshape(TINY.nq, TINY.ntau)
    adj = lambda g: (A.T @ np.ravel(g)).reshape(TINY.nx, TINY.nt)
    return A, fwd, adj, ora


def test_soft_threshold_closed_form():
    v = np.array([-3.0, -1.0, -0.5, -0.2, 0.0, 0.2, 0.5, 1.0, 3.0])
    mu = 1.0  # threshold at mu/2 = 0.5
    np.testing.assert_array_equal(ista.soft_threshold(v, mu),
                                  [-2.5, -0.5, 0.0, 0.0, 0.0, 0.0, 0.0, 0.5, 2.5])
    np.testing.assert_array_equal(ista.soft_threshold(v, 0.0), v)
    np.testing.assert_array_equal(ista.soft_threshold(-v, 0.7), -ista.soft_threshold(v, 0.7))


def test_power_iteration_matches_dense_eigensolver(dense):
    A, fwd, adj, _ = dense
    lam = ista.power_norm2(fwd, adj, (TINY.nx, TINY.nt), iters=400, seed=1)
    ref = np.linalg.eigvalsh(A.T @ A).max()
    assert abs(lam - ref) <= 1e-8 * ref


def test_adjoint_of_dense_operator_is_the_oracle_adjoint(dense):
    A, fwd, adj, ora = dense
    g = np.random.default_rng(3).standard_normal((TINY.nq, TINY.ntau))
    np.testing.assert_allclose(adj(g), ora.adjoint(g), rtol=0, atol=1e-12 * np.abs(adj(g)).max())


@pytest.mark.parametrize("masked", [False, True])
def test_objective_decreases_monotonically(dense, masked):
    A, fwd, adj, _ = dense
    rng = np.random.default_rng(4)
    f = synth.ricker_gather(TINY, 2, 25.0, 7)
    mask = None
    if masked:
        mask = data_mask(TINY, 0.5, 8)
        f = f * mask
    c2 = 0.99 / np.linalg.eigvalsh(A.T @ A).max()
    mu = 0.05 * np.abs(fwd(f)).max()
    g = np.zeros((TINY.nq, TINY.ntau))
    prev = ista.objective(fwd, adj, f, g, mu, mask)
    for _ in range(50):
        g = ista.ista(fwd, adj, f, 1, c2, mu, mask, g0=g)
        cur = ista.objective(fwd, adj, f, g, mu, mask)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_converged_point_satisfies_the_optimality_conditions(dense):
    """Minimiser of ||chi_S(R* g - f)||^2 + mu |g|_1: with r = R chi_S (f - R* g),
    r_i = (mu/2) sign(g_i) where g_i != 0 and |r_i| <= mu/2 where g_i = 0."""
    A, fwd, adj, _ = dense
    f = synth.ricker_gather(TINY, 2, 25.0, 9)
    mask = data_mask(TINY, 0.5, 10)
    f = f * mask
    c2 = 0.99 / np.linalg.eigvalsh(A.T @ A).max()
    mu = 0.1 * np.abs(fwd(f)).max()
    g = ista.ista(fwd, adj, f, 100000, c2, mu, mask)
    r = fwd(mask * (f - adj(g)))
    nz = np.abs(g) > 1e-9 * np.abs(g).max()
    assert nz.any() and (~nz).any()
    tol = 1e-6 * mu
    assert np.all(np.abs(r[nz] - 0.5 * mu * np.sign(g[nz])) <= tol)
    assert np.all(np.abs(r[~nz]) <= 0.5 * mu + tol)


def test_a_planted_sign_error_is_caught(dense):
    """A threshold with the wrong sign of the shift breaks the optimality test."""
    A, fwd, adj, _ = dense
    f = synth.ricker_gather(TINY, 2, 25.0, 9)
    c2 = 0.99 / np.linalg.eigvalsh(A.T @ A).max()
    mu = 0.1 * np.abs(fwd(f)).max()
    g = np.zeros((TINY.nq, TINY.ntau))
    for _ in range(3000):
        v = g + c2 * fwd(f - adj(g))
        h = 0.5 * c2 * mu
        g = np.where(v >= h, v + h, np.where(v <= -h, v - h, 0.0))  # wrong sign
    r = fwd(f - adj(g))
    nz = np.abs(g) > 0
    assert not np.all(np.abs(r[nz] - 0.5 * mu * np.sign(g[nz])) <= 1e-6 * mu)
