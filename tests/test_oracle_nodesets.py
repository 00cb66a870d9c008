"""Pins of the node sets beyond the paper's trapezoid and Simpson methods
(paper Sec. 5: other quadratures for highly stiff reactions): Gauss-Lobatto
with 4 and 5 nodes and right Radau (Radau IIA) points.

What fixes them, independently of the oracle's own code:
* the classical Radau IIA tableaux (tests/golden/radau_iia.txt);
* the fixed point of the sweeps on a linear system x' = L x is the method's
  stability function applied to dt L: the diagonal Pade approximant (s-1, s-1)
  of exp for s Lobatto nodes (Lobatto IIIA) and the subdiagonal (s-1, s) for s
  Radau points (Radau IIA), from the textbook Pade formula;
* L-stability of Radau IIA: a stiff transient is damped in one large step,
  where Lobatto IIIA carries it over undamped;
* the measured order of accuracy against expm(L t) x0.
"""
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla

import sdc_inputs as si
from oracle import quadrature, sdc
from tests import golden
from tests.test_oracle_sdc import chain_operator

G = golden.read("radau_iia.txt")


@pytest.mark.parametrize("s", [1, 2, 3])
def test_radau_points_and_collocation_matrix_are_radau_iia(s):
    tau, S = quadrature.node_set("radau", s + 1)
    np.testing.assert_allclose(tau[0], 0.0)
    np.testing.assert_allclose(tau[1:], G[f"c{s}"], atol=2e-16)
    assert np.all(S[:, 0] == 0.0)  # node 0 is not an interpolation point
    A = np.cumsum(S, axis=0)[:, 1:]  # a_ij = int_0^{c_i} l_j
    for i in range(s):
        np.testing.assert_allclose(A[i], G[f"A{s}_row{i}"], atol=3e-16)


@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_radau_subinterval_weights_exact_to_degree_s_minus_1(s):
    tau, S = quadrature.node_set("radau", s + 1)
    for p in range(s):
        exact = (tau[1:] ** (p + 1) - tau[:-1] ** (p + 1)) / (p + 1)
        np.testing.assert_allclose(S @ tau ** p, exact, atol=1e-14)
    p = s
    exact = (tau[1:] ** (p + 1) - tau[:-1] ** (p + 1)) / (p + 1)
    assert np.max(np.abs(S @ tau ** p - exact)) > 1e-6


def pade_exp(k, m, Z):
    """The (k, m) Pade approximant of exp at the matrix Z: Q(Z)^{-1} P(Z) with
    P(z) = sum_j (k+m-j)! k! / ((k+m)! j! (k-j)!) z^j and
    Q(z) = sum_j (k+m-j)! m! / ((k+m)! j! (m-j)!) (-z)^j."""
    n = Z.shape[0]
    P = np.zeros((n, n))
    Q = np.zeros((n, n))
    Zj = np.eye(n)
    for j in range(max(k, m) + 1):
        if j <= k:
            P += factorial(k + m - j) * factorial(k) / (factorial(k + m) * factorial(j) * factorial(k - j)) * Zj
        if j <= m:
            Q += factorial(k + m - j) * factorial(m) / (factorial(k + m) * factorial(j) * factorial(m - j)) * (-1) ** j * Zj
        Zj = Zj @ Z
    return np.linalg.solve(Q, P)


def chain_problem(**over):
    w = si.workload("chain1d")
    return w, sdc.Problem.from_workload(w, advection=0, **over)


@pytest.mark.parametrize("kind,n_nodes,k,m", [("lobatto", 4, 3, 3), ("lobatto", 5, 4, 4), ("radau", 2, 0, 1),
                                               ("radau", 3, 1, 2), ("radau", 4, 2, 3), ("radau", 5, 3, 4)])
def test_fixed_point_is_the_pade_approximant(kind, n_nodes, k, m):
    """Iterated to convergence on the stiff linear chain (rates 1, 1e3, 1e6,
    dt = 1e-4), one step equals the method's stability function at dt L."""
    w, p = chain_problem(n_nodes=n_nodes, node_type=kind, n_iters=80)
    dt = 1e-4
    U1, _, _ = sdc.step(w["U0"], dt, p)
    _, _, x0, _ = sdc.split_state(w["U0"], p)
    _, _, x1, _ = sdc.split_state(U1, p)
    ref = pade_exp(k, m, dt * chain_operator(p.net)) @ x0
    err = np.max(np.abs(x1 - ref)) / np.max(np.abs(ref))
    print(f"{kind} {n_nodes} nodes: fixed point vs Pade ({k},{m}): {err:.2e}")
    assert err < 1e-13


def test_radau_damps_a_stiff_transient_lobatto_does_not():
    """L-stability: species C of the chain decays at rate 1e6; started far from
    its quasi-steady state, one step of dt = 1e-3 (dt * 1e6 = 1000) at the
    fixed point leaves it within 1% of the exact value with Radau points (R(-inf) = 0),
    while the Lobatto IIIA fixed point keeps the transient (R(-inf) = 1)."""
    net = si.chain_network()
    dt = 1e-3
    x0 = np.array([0.5, 0.3, 0.2, 0.0, 1.0])  # rho X_A..X_D, rho e
    Lop = chain_operator(net)
    exact = sla.expm(Lop * dt) @ x0
    out = {}
    for kind, n in (("radau", 3), ("lobatto", 3)):
        w, p = chain_problem(n_nodes=n, node_type=kind, n_iters=200)
        U0 = w["U0"].copy()
        rho, mom, _, ke = sdc.split_state(U0, p)
        x = np.repeat(x0[:, None], rho.size, axis=1) * rho[None]
        x[4] = x0[4] * rho
        U0 = sdc.join_state(rho, mom, x, ke, p)
        U1, _, _ = sdc.step(U0, dt, p)
        _, _, x1, _ = sdc.split_state(U1, p)
        out[kind] = np.max(np.abs(x1[2] / rho - exact[2]))
    print(f"stiff species error: radau {out['radau']:.2e}, lobatto {out['lobatto']:.2e}")
    assert out["radau"] < 1e-2 * x0[2]  # |R(z)| = O(1/|z|) at z = -1000
    assert out["lobatto"] > 0.5 * x0[2]


@pytest.mark.parametrize("kind,n_nodes,K,order,steps", [("lobatto", 4, 6, 5.7, (2, 4, 8, 16)),
                                                        ("lobatto", 5, 8, 7.5, (1, 2, 4, 8)),
                                                        ("radau", 3, 6, 2.9, (4, 8, 16, 32)),
                                                        ("radau", 4, 10, 4.9, (4, 8, 16, 32))])
def test_measured_order_against_the_exponential(kind, n_nodes, K, order, steps):
    """A non-stiff chain (rates 1, 2, 3) against expm(L T) x0 over T = 1: the
    error falls at the design order, 2M for M + 1 Lobatto nodes (orders 6 and 8
    with K = 2M sweeps) and 2s - 1 for s Radau points (orders 3 and 5, with
    enough sweeps to reach the collocation solution's order); step counts keep
    the finest error above rounding."""
    net = si.chain_network(rates=(1.0, 2.0, 3.0))
    w, p = chain_problem(n_nodes=n_nodes, node_type=kind, n_iters=K)
    p.net = net
    Tf = 1.0
    _, _, x0, _ = sdc.split_state(w["U0"], p)
    ref = sla.expm(chain_operator(net) * Tf) @ x0
    errs = []
    for nst in steps:
        U = sdc.run(w["U0"], Tf / nst, nst, p)
        _, _, x1, _ = sdc.split_state(U, p)
        errs.append(np.max(np.abs(x1 - ref)) / np.max(np.abs(ref)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    print(f"{kind} {n_nodes} nodes K={K}: errors {errs}, rates {rates}")
    assert errs[-1] > 1e-14  # above rounding, so the rate is measured
    assert rates[-1] > order, rates
