"""Pins P2-P7 of the oracle's SDC step (paper Sec. 2, Eq. 2)."""
import dataclasses

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.integrate import solve_ivp

import sdc_inputs as si
from oracle import network, sdc

GAMMA = 1.4


def chain_operator(net):
    """The chain as a linear system on (x_s, x_e): x' = L x."""
    ns = net["nspec"]
    k = np.exp(net["lnA"])
    L = np.zeros((ns + 1, ns + 1))
    for r in range(net["nreact"]):
        L[r, r] -= k[r]
        L[r + 1, r] += k[r]
    L[ns, :ns] = -net["q"] @ L[:ns, :ns]
    return L


def _chain(**over):
    w = si.workload("chain1d")
    return w, sdc.Problem.from_workload(w, **over)


@pytest.mark.parametrize("n_nodes", [2, 3])
def test_fixed_point_is_the_pade_approximant(n_nodes):
    """P2: iterated to convergence, Eq. 2 becomes Lobatto IIIA collocation, whose
    stability function on x' = L x is the diagonal Pade approximant (1,1) for
    2 nodes and (2,2) for 3 nodes.  Stiff rates (1, 1e3, 1e6), dt = 1e-3."""
    w, p = _chain(n_nodes=n_nodes, n_iters=60, advection=0)
    dt = 1e-3
    U1, _, _ = sdc.step(w["U0"], dt, p)
    _, _, x0, _ = sdc.split_state(w["U0"], p)
    _, _, x1, _ = sdc.split_state(U1, p)
    Z = dt * chain_operator(p.net)
    I = np.eye(5)
    if n_nodes == 2:
        P = np.linalg.solve(I - Z / 2, I + Z / 2)
    else:
        P = np.linalg.solve(I - Z / 2 + Z @ Z / 12, I + Z / 2 + Z @ Z / 12)
    ref = P @ x0
    assert np.max(np.abs(x1 - ref)) / np.max(np.abs(ref)) < 1e-15


def test_first_sweep_is_backward_euler_between_nodes():
    """P3: with K = 1 and A = 0 the iteration-0 reading makes the sweep a
    backward-Euler step per sub-interval."""
    dt = 2e-3
    _, _, x0, _ = sdc.split_state(_chain()[0]["U0"], _chain()[1])
    for n_nodes, subs in [(2, [1.0]), (3, [0.5, 0.5])]:
        w, p = _chain(n_nodes=n_nodes, n_iters=1, advection=0)
        U1, _, _ = sdc.step(w["U0"], dt, p)
        _, _, x1, _ = sdc.split_state(U1, p)
        L = chain_operator(p.net)
        ref = x0
        for f in subs:
            ref = np.linalg.solve(np.eye(5) - f * dt * L, ref)
        assert np.max(np.abs(x1 - ref)) / np.max(np.abs(ref)) < 1e-14


def test_first_sweep_with_advection_is_imex_euler():
    """P3 with A != 0: U^{1} = U^n + dt A(U^n) + dt R(U^{1}) for 2 nodes, K = 1."""
    w, p = _chain(n_nodes=2, n_iters=1)
    dt = w["dt"]
    U0 = w["U0"]
    U1, _, _ = sdc.step(U0, dt, p)
    rhs = U0 + dt * sdc.A_of(U0, p)
    rho, mom, b, ke = sdc.split_state(rhs, p)
    L = chain_operator(p.net)
    x = np.linalg.solve(np.eye(5) - dt * L, b)
    ref = sdc.join_state(rho, mom, x, ke, p)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.max(np.abs(U1 - ref) / scale) < 1e-14


@pytest.mark.parametrize("n_nodes,K,order", [(2, 2, 1.9), (3, 4, 3.8)])
def test_linear_chain_converges_to_exponential_at_design_order(n_nodes, K, order):
    """P4/P5: A = 0 chain vs the closed form expm(L t) x0 (stiff rates), error
    at rate dt^{min(K, 2M)}; the energy released is part of x."""
    w, p = _chain(n_nodes=n_nodes, n_iters=K, advection=0)
    Tf = 1e-3
    _, _, x0, _ = sdc.split_state(w["U0"], p)
    ref = sla.expm(chain_operator(p.net) * Tf) @ x0
    errs = []
    for nst in (8, 16, 32, 64):
        U = sdc.run(w["U0"], Tf / nst, nst, p)
        _, _, x1, _ = sdc.split_state(U, p)
        errs.append(np.max(np.abs(x1 - ref)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1] > order, rates
    assert np.all(rates > order - 0.5), rates


@pytest.mark.parametrize("n_nodes,K,order", [(2, 2, 1.85), (3, 4, 3.8), (3, 30, 3.95)])
def test_nonlinear_network_against_radau(n_nodes, K, order):
    """P6: A = 0, a non-stiff seeded Arrhenius network, sampled zones against
    scipy's Radau IIA at rtol 1e-13 (independent brute force)."""
    w = si.workload("net2d", shape=(8, 8))
    net = si.random_network(7, 10, 77, log10A=(1.0, 2.0), E=(1.0, 3.0))
    p = sdc.Problem.from_workload(w, advection=0, net=net, n_nodes=n_nodes, n_iters=K)
    rho, _, x0, _ = sdc.split_state(w["U0"], p)
    zs = np.arange(0, 64, 9)
    Tf = 0.05

    def f(t, y, z):
        return network.source(y[:, None], rho[z:z + 1], net, GAMMA)[:, 0]

    def jac(t, y, z):
        return network.source_and_jacobian(y[:, None], rho[z:z + 1], net, GAMMA)[1][0]

    ref = np.stack([solve_ivp(f, (0, Tf), x0[:, z], method="Radau", rtol=1e-13, atol=1e-15,
                              jac=jac, args=(z,)).y[:, -1] for z in zs], axis=1)
    ns = net["nspec"]
    sc = np.concatenate([np.broadcast_to(rho[zs], (ns, zs.size)), np.abs(ref[ns:])])
    errs = []
    for nst in (2, 4, 8, 16):
        U = sdc.run(w["U0"], Tf / nst, nst, p)
        _, _, x1, _ = sdc.split_state(U, p)
        errs.append(np.max(np.abs(x1[:, zs] - ref) / sc))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1] > order, (errs, rates)
    assert errs[-1] < 1e-3


@pytest.mark.parametrize("n_nodes,K,order", [(2, 2, 1.9), (3, 4, 3.7)])
def test_coupled_hydro_reaction_temporal_order(n_nodes, K, order):
    """P5 with A != 0: the chain with smooth-mode advection, self-convergence
    against a 16x finer step than the finest on the same grid (method of lines, so the spatial
    error cancels)."""
    w = si.workload("chain1d")
    net = si.chain_network(rates=(1.0, 30.0, 1.0e3))
    p = sdc.Problem.from_workload(w, n_nodes=n_nodes, n_iters=K, slope=0, alpha=2.0, net=net)
    Tf = 4 * w["dt"]
    ref = sdc.run(w["U0"], Tf / 512, 512, p)
    errs = []
    for nst in (4, 8, 16, 32):
        U = sdc.run(w["U0"], Tf / nst, nst, p)
        errs.append(np.max(np.abs(U - ref) / np.abs(ref).max(axis=1, keepdims=True)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert rates[-1] > order, (errs, rates)


@pytest.mark.parametrize("slope", [0, 1])
def test_global_conservation_over_steps(slope):
    """P7 (iii): sum_z rho, sum_z rho u and sum_z (rho E + sum_i q_i rho X_i) are
    constant; with central slopes (and A = 0) each zone's species sum stays rho."""
    w = si.workload("net2d", shape=(16, 16))
    p = sdc.Problem.from_workload(w, slope=slope, alpha=(1.7 if slope == 0 else -1.0))
    U0 = w["U0"]
    U = sdc.run(U0, 0.5 * w["dt"], 2, p)
    d, q = p.dim, p.net["q"]

    def invariants(V):
        Vf = V.reshape(V.shape[0], -1)
        return np.array([Vf[0].sum(), Vf[1].sum(), Vf[2].sum(),
                         (Vf[1 + d] + q @ Vf[2 + d:]).sum()])

    i0, i1 = invariants(U0), invariants(U)
    scale = np.array([i0[0], np.abs(U0[1]).sum(), np.abs(U0[2]).sum(), i0[3]])
    assert np.max(np.abs(i1 - i0) / scale) < 2e-14
    if slope == 0:
        Uf = U.reshape(U.shape[0], -1)
        assert np.max(np.abs(Uf[2 + d:].sum(0) - Uf[0]) / Uf[0]) < 1e-13
    # the step really burned something
    assert np.max(np.abs(U[2 + d] - U0[2 + d])) > 1e-6


def test_sweep_stats_are_recorded():
    w = si.workload("net2d", shape=(8, 8))
    p = sdc.Problem.from_workload(w)
    st = sdc.Stats()
    sdc.step(w["U0"], w["dt"], p, stats=st)
    assert st.solves == 64 * 2 * 4 and st.failed == 0
    assert st.hist.sum() == st.solves and st.newton_total == (st.hist * np.arange(16)).sum()
