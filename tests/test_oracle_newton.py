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


def test_rate_stop_returns_roots_within_the_tolerance():
    """The stopping test on the contraction of successive steps returns
    iterates within tol (scaled as the steps are) of the root that three more
    Newton steps reach, on the stiff networks at the workload's step and at
    10 and 100 times it."""
    for name, shape in (("net3d", (6, 5, 4)), ("net2d", (12, 10))):
        w = si.workload(name, shape=shape)
        p = sdc.Problem.from_workload(w, advection=0)
        rho, _, x0, _ = sdc.split_state(w["U0"], p)
        g = si.rng(3)
        ns = p.nspec
        for f in (1, 10, 100):
            dt = f * w["dt"]
            b = x0 * (1 + 0.05 * g.uniform(-1, 1, x0.shape))
            x, _, nu = sdc.reaction_solve(dt, rho, b, x0, p)
            xe, _, _ = sdc.reaction_solve(dt, rho, b, x0, dataclasses.replace(p, newton_extra=3))
            scale = np.concatenate([np.broadcast_to(rho, (ns, rho.size)), np.abs(b[ns])[None]])
            dist = np.max(np.abs(x - xe) / scale, axis=0)
            assert np.all(nu > 0)
            assert dist.max() <= p.newton_tol, (name, f, dist.max())


def test_rate_stop_count_from_the_iterates():
    """The iteration at which each solve stops, recounted from the Newton
    iterates themselves: runs of exactly j steps (tol = 0, maxiter = j) give
    x_j, the step sizes e_j are their scaled differences, and the solve must
    stop at the first j with e_j <= tol or e_j^2 <= tol (e_{j-1} - e_j),
    e_j < e_{j-1} (the stopping rule as stated; this checks its bookkeeping:
    which step is compared with which, the scaling, the first step)."""
    w = si.workload("net2d", shape=(6, 5))
    p = sdc.Problem.from_workload(w, advection=0)
    rho, _, x0, _ = sdc.split_state(w["U0"], p)
    ns = p.nspec
    dt = 30 * w["dt"]
    b = x0 * (1 + 0.05 * si.rng(5).uniform(-1, 1, x0.shape))
    _, _, nu = sdc.reaction_solve(dt, rho, b, x0, p)
    scale = np.concatenate([np.broadcast_to(rho, (ns, rho.size)), np.abs(b[ns])[None]])
    xs = [x0] + [sdc.reaction_solve(dt, rho, b, x0, dataclasses.replace(p, newton_tol=0.0, newton_maxiter=j))[0]
                 for j in range(1, nu.max() + 1)]
    e = [np.max(np.abs(xs[j] - xs[j - 1]) / scale, axis=0) for j in range(1, len(xs))]
    tol = p.newton_tol
    expect = np.zeros_like(nu)
    for z in range(nu.size):
        for j in range(len(e)):
            ej, ep = e[j][z], (e[j - 1][z] if j else 0.0)
            if ej <= tol or (ej < ep and ej * ej <= tol * (ep - ej)):
                expect[z] = j + 1
                break
    assert np.all(nu == expect), (nu, expect)
    assert np.any(np.array([e[n - 1][z] for z, n in enumerate(nu)]) > tol)  # the rate test decided some
