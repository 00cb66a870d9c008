"""Temporal nodes and the node-to-node integration matrix (oracle).

Eq. 2 of the paper needs, for every pair of neighbouring nodes, the integral
from t^m to t^{m+1} of the previous iteration's sources, built from the values
at all nodes (Sec. 2).  The paper names the trapezoid rule (2nd-order method)
and Simpson's rule (4th-order method).  Reading: the nodes are Gauss-Lobatto
points on [0, 1] ({0, 1} and {0, 1/2, 1}) and the node-to-node integral is the
exact integral of the Lagrange interpolant through all nodes; summed over the
sub-intervals this is the trapezoid / Simpson rule.

The paper's outlook (Sec. 5) names other quadratures, better suited to highly
stiff reactions, as the next step.  Reading: Radau IIA points, the right
Radau points on (0, 1] (end point 1 included).  The node list is then tau_0 = 0
(the step's initial value, which is not a quadrature point) followed by the s
Radau points, and the integrand is interpolated through the s Radau points
only, so column 0 of S is zero.  The fixed point of the sweeps is then the
s-stage Radau IIA collocation solution (L-stable), where the Gauss-Lobatto set
gives Lobatto IIIA (A-stable, no damping at infinite stiffness).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as P


def gauss_lobatto_nodes(n_nodes: int) -> np.ndarray:
    """Gauss-Lobatto points on [0, 1]: the end points plus the roots of P'_{n-1}."""
    if n_nodes < 2:
        raise ValueError("need at least 2 nodes")
    if n_nodes == 2:
        inner = np.array([])
    else:
        c = np.zeros(n_nodes)
        c[-1] = 1.0  # P_{n-1}
        inner = np.sort(L.legroots(L.legder(c)).real)
    s = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (s + 1.0)


def radau_right_nodes(n_nodes: int) -> np.ndarray:
    """0 followed by the s = n_nodes - 1 right Radau points on (0, 1]: the
    zeros of P_s(2t - 1) - P_{s-1}(2t - 1), whose largest is t = 1."""
    s = n_nodes - 1
    if s < 1:
        raise ValueError("need at least 2 nodes")
    c = np.zeros(s + 1)
    c[s] = 1.0
    c[s - 1] = -1.0  # P_s - P_{s-1}
    y = np.sort(L.legroots(c).real)
    y[-1] = 1.0  # exact root
    return np.concatenate([[0.0], 0.5 * (y + 1.0)])


def nodes(kind: str, n_nodes: int) -> np.ndarray:
    """Node list of a step on [0, 1] for kind 'lobatto' or 'radau'."""
    if kind == "lobatto":
        return gauss_lobatto_nodes(n_nodes)
    if kind == "radau":
        return radau_right_nodes(n_nodes)
    raise ValueError(f"unknown node kind {kind!r}")


def lagrange_basis(tau: np.ndarray, j: int) -> np.ndarray:
    """Power-series coefficients of the Lagrange polynomial l_j through tau."""
    coef = np.array([1.0])
    for i, ti in enumerate(tau):
        if i != j:
            coef = P.polymul(coef, np.array([-ti, 1.0]) / (tau[j] - ti))
    return coef


def integration_matrix(tau: np.ndarray, first: int = 0) -> np.ndarray:
    """S[m, j] = int_{tau_m}^{tau_{m+1}} l_j(s) ds on the unit interval, with
    l_j the Lagrange polynomials through the interpolation points
    tau[first:] (columns j < first are zero).

    For a step of length dt, int_{t^m}^{t^{m+1}} f dt ~= dt * sum_j S[m, j] f_j.
    """
    n = len(tau)
    pts = tau[first:]
    S = np.zeros((n - 1, n))
    for j in range(first, n):
        anti = P.polyint(lagrange_basis(pts, j - first))
        for m in range(n - 1):
            S[m, j] = P.polyval(tau[m + 1], anti) - P.polyval(tau[m], anti)
    return S


def node_set(kind: str, n_nodes: int):
    """(tau, S) of a node kind: Gauss-Lobatto interpolates through every
    node, Radau through the Radau points (all nodes but tau_0 = 0)."""
    tau = nodes(kind, n_nodes)
    return tau, integration_matrix(tau, first=0 if kind == "lobatto" else 1)
