"""Temporal nodes and the node-to-node integration matrix (oracle).

Eq. 2 of the paper needs, for every pair of neighbouring nodes, the integral
from t^m to t^{m+1} of the previous iteration's sources, built from the values
at all nodes (Sec. 2).  The paper names the trapezoid rule (2nd-order method)
and Simpson's rule (4th-order method).  Reading: the nodes are Gauss-Lobatto
points on [0, 1] ({0, 1} and {0, 1/2, 1}) and the node-to-node integral is the
exact integral of the Lagrange interpolant through all nodes; summed over the
sub-intervals this is the trapezoid / Simpson rule.
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


def lagrange_basis(tau: np.ndarray, j: int) -> np.ndarray:
    """Power-series coefficients of the Lagrange polynomial l_j through tau."""
    coef = np.array([1.0])
    for i, ti in enumerate(tau):
        if i != j:
            coef = P.polymul(coef, np.array([-ti, 1.0]) / (tau[j] - ti))
    return coef


def integration_matrix(tau: np.ndarray) -> np.ndarray:
    """S[m, j] = int_{tau_m}^{tau_{m+1}} l_j(s) ds on the unit interval.

    For a step of length dt, int_{t^m}^{t^{m+1}} f dt ~= dt * sum_j S[m, j] f_j.
    """
    n = len(tau)
    S = np.zeros((n - 1, n))
    for j in range(n):
        anti = P.polyint(lagrange_basis(tau, j))
        for m in range(n - 1):
            S[m, j] = P.polyval(tau[m + 1], anti) - P.polyval(tau[m], anti)
    return S
