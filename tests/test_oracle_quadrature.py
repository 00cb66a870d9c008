"""Pin P1: nodes and node-to-node quadrature of the oracle (paper Sec. 2)."""
import numpy as np
import pytest

from oracle import quadrature
from tests import golden

G = golden.read("gauss_lobatto.txt")


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_gauss_lobatto_points_match_classical_values(n):
    np.testing.assert_allclose(quadrature.gauss_lobatto_nodes(n), G[f"nodes{n}"], atol=1e-15)


def test_sub_interval_weights_classical():
    S2 = quadrature.integration_matrix(quadrature.gauss_lobatto_nodes(2))
    S3 = quadrature.integration_matrix(quadrature.gauss_lobatto_nodes(3))
    np.testing.assert_allclose(S2[0], G["S2_row0"], atol=1e-15)
    np.testing.assert_allclose(S3[0], G["S3_row0"], atol=1e-15)
    np.testing.assert_allclose(S3[1], G["S3_row1"], atol=1e-15)
    # summed over the sub-intervals: trapezoid and Simpson on the whole step
    np.testing.assert_allclose(S2.sum(axis=0), [0.5, 0.5], atol=1e-15)
    np.testing.assert_allclose(S3.sum(axis=0), [1 / 6, 4 / 6, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_exact_on_polynomials_up_to_degree_n_minus_1(n):
    tau = quadrature.gauss_lobatto_nodes(n)
    S = quadrature.integration_matrix(tau)
    for p in range(n):
        exact = (tau[1:] ** (p + 1) - tau[:-1] ** (p + 1)) / (p + 1)
        np.testing.assert_allclose(S @ tau ** p, exact, atol=1e-14)
    # and not exact one degree higher on some sub-interval (the order is sharp)
    p = n
    exact = (tau[1:] ** (p + 1) - tau[:-1] ** (p + 1)) / (p + 1)
    assert np.max(np.abs(S @ tau ** p - exact)) > 1e-6
