"""Pins of the oracle's implicit reaction solve (the implicit part of Eq. 2)."""
import dataclasses

import numpy as np

import sdc_inputs as si
from oracle import sdc

GAMMA = 1.4


def _problem(name):
    w = si.workload(name, shape=(8,) if name == "chain1d" else (8, 8))
    return w, sdc.Problem.from_workload(w, advection=0)


def test_linear_chain_solve_is_the_direct_linear_solve():
    """For constant rates x - dt K x = b has the unique root (I - dt K)^{-1} b."""
    w, p = _problem("chain1d")
    rho, _, x0, _ = sdc.split_state(w["U0"], p)
    g = si.rng(9)
    b = x0 * (1 + 0.1 * g.uniform(-1, 1, x0.shape))
    dt = 2e-3
    x, R, nu = sdc.reaction_solve(dt, rho, b, x0, p)
    k = [1.0, 1.0e3, 1.0e6]
    K = np.zeros((5, 5))
    for r in range(3):
        K[r, r] -= k[r]
        K[r + 1, r] += k[r]
    K[4, :4] = -p.net["q"] @ K[:4, :4]
    ref = np.linalg.solve(np.eye(5) - dt * K, b)
    np.testing.assert_allclose(x, ref, rtol=1e-13, atol=1e-15)
    assert np.all(nu == 2)  # exact after one step; the second confirms |delta| <= tol


def test_nonlinear_root_residual_and_conservation():
    w, p = _problem("net2d")
    rho, _, x0, _ = sdc.split_state(w["U0"], p)
    b = x0.copy()
    dt = 3e-3
    x, R, nu = sdc.reaction_solve(dt, rho, b, x0, p)
    assert np.all(nu > 0) and np.all(nu < 12)
    G = x - dt * R - b
    ns = p.nspec
    assert np.max(np.abs(G[:ns]) / rho) < 1e-14
    assert np.max(np.abs(G[ns]) / np.abs(b[ns])) < 1e-14
    # P7 (i): mass sum is conserved by the solve, (ii): energy invariant
    assert np.max(np.abs(x[:ns].sum(0) - b[:ns].sum(0)) / rho) < 1e-14
    q = p.net["q"]
    inv_x = x[ns] + q @ x[:ns]
    inv_b = b[ns] + q @ b[:ns]
    assert np.max(np.abs(inv_x - inv_b) / np.abs(inv_b)) < 1e-14
    # and the reaction actually did something
    assert np.max(np.abs(x[:ns] - b[:ns]) / rho) > 1e-3


def test_failure_reports_minus_one_and_keeps_last_iterate():
    w, p = _problem("net2d")
    p1 = dataclasses.replace(p, newton_maxiter=1)
    rho, _, x0, _ = sdc.split_state(w["U0"], p)
    x, R, nu = sdc.reaction_solve(3e-3, rho, x0.copy(), x0, p1)
    assert np.all(nu == -1)
    # the kept iterate is one Newton step from x0: compare against maxiter=1 by hand
    x2, _, nu2 = sdc.reaction_solve(3e-3, rho, x0.copy(), x, p)
    assert np.all(nu2 > 0)
    assert np.max(np.abs(x - x0) / rho) > 0
