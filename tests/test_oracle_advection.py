"""Pin P8: invariants and spatial order of the oracle's advective term."""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import advection

GAMMA = 1.4


def _smooth_2d(nx, ny, nspec=3, seed=3):
    g = si.rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    Y, X = np.meshgrid(y, x, indexing="ij")
    ph = g.uniform(0, 1, 6)
    rho = 1 + 0.2 * np.sin(2 * np.pi * (X + ph[0])) * np.cos(2 * np.pi * (Y + ph[1]))
    u = [0.3 * np.sin(2 * np.pi * (Y + ph[2])), 0.2 * np.cos(2 * np.pi * (X + ph[3]))]
    p = 1 + 0.1 * np.sin(2 * np.pi * (X + Y + ph[4]))
    Xs = g.uniform(0.1, 1, (nspec,) + rho.shape)
    Xs /= Xs.sum(0)
    return si.conserved_from_primitive(rho, u, p, Xs)


@pytest.mark.parametrize("slope", [0, 1])
def test_uniform_state_gives_exactly_zero(slope):
    U = _smooth_2d(8, 8)
    U[:] = U[:, :1, :1]
    A = advection.advective_term(U, 2, [1 / 8, 1 / 8], GAMMA, slope)
    assert np.all(A == 0.0)


@pytest.mark.parametrize("slope,alpha", [(0, -1.0), (1, -1.0), (0, 1.7)])
def test_periodic_sum_vanishes(slope, alpha):
    U = _smooth_2d(16, 12)
    A = advection.advective_term(U, 2, [1 / 16, 1 / 12], GAMMA, slope, alpha)
    assert np.max(np.abs(A.sum(axis=(1, 2)))) < 1e-12 * np.abs(A).max() * A[0].size


@pytest.mark.parametrize("slope", [0, 1])
def test_y_invariant_2d_equals_1d(slope):
    U2 = _smooth_2d(16, 8)
    U2[:] = U2[:, :1, :]
    U2[2] = 0.0  # no y momentum
    A2 = advection.advective_term(U2, 2, [1 / 16, 1 / 8], GAMMA, slope)
    U1 = np.delete(U2[:, 0, :], 2, axis=0)
    A1 = advection.advective_term(U1, 1, [1 / 16], GAMMA, slope)
    assert np.array_equal(np.delete(A2[:, 0, :], 2, axis=0), A1)
    assert np.all(A2[2] == 0.0)
    assert np.array_equal(A2[:, 3, :], A2[:, 0, :])


@pytest.mark.parametrize("slope", [0, 1])
def test_axis_permutation_transposes_result(slope):
    U = _smooth_2d(12, 12)
    A = advection.advective_term(U, 2, [1 / 12, 1 / 12], GAMMA, slope)
    Ut = U.transpose(0, 2, 1).copy()
    Ut[[1, 2]] = Ut[[2, 1]]  # swap momentum components with the axes
    At = advection.advective_term(Ut, 2, [1 / 12, 1 / 12], GAMMA, slope)
    At[[1, 2]] = At[[2, 1]]
    assert np.array_equal(At.transpose(0, 2, 1), A)


def _advection_error(n, slope, norm):
    """Uniform u and p: the exact divergence is -u d(rho)/dx, -u d(rho X)/dx."""
    x = (np.arange(n) + 0.5) / n
    rho = 1 + 0.3 * np.sin(2 * np.pi * x)
    u, p = 0.7, 1.0
    Xs = np.stack([0.6 + 0.2 * np.cos(2 * np.pi * x), 0.4 - 0.2 * np.cos(2 * np.pi * x)])
    U = si.conserved_from_primitive(rho, [np.full(n, u)], np.full(n, p), Xs)
    A = advection.advective_term(U, 1, [1 / n], GAMMA, slope)
    drho = 0.6 * np.pi * np.cos(2 * np.pi * x)
    dX0 = -0.4 * np.pi * np.sin(2 * np.pi * x)
    exact_rho = -u * drho
    exact_s0 = -u * (drho * Xs[0] + rho * dX0)
    exact_mom = -u * u * drho
    err = np.concatenate([A[0] - exact_rho, A[1] - exact_mom, A[3] - exact_s0])
    return np.max(np.abs(err)) if norm == "max" else np.mean(np.abs(err))


@pytest.mark.parametrize("slope,norm,order", [(0, "max", 1.95), (1, "l1", 1.9)])
def test_second_order_in_space(slope, norm, order):
    e = np.array([_advection_error(n, slope, norm) for n in (64, 128, 256)])
    rates = np.log2(e[:-1] / e[1:])
    assert np.all(rates > order), rates
