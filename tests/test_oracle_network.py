"""Pins of the oracle's synthetic network: analytic Jacobian (P9), exact
conservation identities (P7) and the linear-chain special case."""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import network

GAMMA = 1.4


def _state(net, Z=17, seed=5):
    g = si.rng(seed)
    ns = net["nspec"]
    rho = g.uniform(0.7, 1.4, Z)
    X = g.uniform(0.0, 1.0, (ns, Z))
    X /= X.sum(axis=0)
    T = g.uniform(0.8, 1.3, Z)
    x = np.concatenate([rho * X, (rho * T / (GAMMA - 1))[None]])
    return x, rho


NETS = {
    "chain": si.chain_network(),
    "net7": si.random_network(7, 10, si.SEEDS["net7_network"]),
    "net13": si.random_network(13, 20, si.SEEDS["net13_network"]),
}


@pytest.mark.parametrize("name", list(NETS))
def test_jacobian_matches_complex_step(name):
    net = NETS[name]
    x, rho = _state(net)
    R, J = network.source_and_jacobian(x, rho, net, GAMMA)
    n = x.shape[0]
    h = 1e-30
    for j in range(n):
        xc = x.astype(complex)
        step = h * np.abs(x[j]).max()
        xc[j] += 1j * step
        col = network.source(xc, rho, net, GAMMA).imag / step
        scale = np.abs(J).max(axis=(1, 2))
        err = np.abs(col.T - J[:, :, j]) / scale[:, None]
        assert err.max() < 1e-13, (name, j, err.max())
    np.testing.assert_allclose(R, network.source(x, rho, net, GAMMA), rtol=0, atol=0)


@pytest.mark.parametrize("name", list(NETS))
def test_parameter_derivatives_match_complex_step(name):
    net = NETS[name]
    x, rho = _state(net)
    dlnA, dE = network.source_param_derivatives(x, rho, net, GAMMA)
    h = 1e-30
    for r in range(net["nreact"]):
        lnA = net["lnA"].astype(complex)
        lnA[r] += 1j * h
        g = network.source(x, rho, net, GAMMA, lnA=lnA).imag / h
        np.testing.assert_allclose(g, dlnA[r], rtol=1e-13, atol=1e-300)
        E = net["E"].astype(complex)
        E[r] += 1j * h
        g = network.source(x, rho, net, GAMMA, E=E).imag / h
        np.testing.assert_allclose(g, dE[r], rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("name", list(NETS))
def test_mass_and_energy_identities(name):
    """sum_i R_i = 0 (mass) and R_e + sum_i q_i R_i = 0 (energy), exactly up to
    rounding, and the same for every Jacobian column."""
    net = NETS[name]
    x, rho = _state(net)
    R, J = network.source_and_jacobian(x, rho, net, GAMMA)
    ns = net["nspec"]
    scale = np.abs(R).max(axis=0)
    assert np.max(np.abs(R[:ns].sum(axis=0)) / scale) < 1e-14
    assert np.max(np.abs(R[ns] + net["q"] @ R[:ns]) / scale) < 1e-14
    jscale = np.abs(J).max()
    assert np.max(np.abs(J[:, :ns, :].sum(axis=1))) / jscale < 1e-14
    assert np.max(np.abs(J[:, ns, :] + np.einsum("i,zij->zj", net["q"], J[:, :ns, :]))) / jscale < 1e-14


def test_chain_is_the_textbook_linear_system():
    """With constant rates the chain is x' = K x with the bidiagonal matrix of
    A->B->C->D, independent of T."""
    net = NETS["chain"]
    x, rho = _state(net)
    k = [1.0, 1.0e3, 1.0e6]
    K = np.array([[-k[0], 0, 0, 0],
                  [k[0], -k[1], 0, 0],
                  [0, k[1], -k[2], 0],
                  [0, 0, k[2], 0]])
    R = network.source(x, rho, net, GAMMA)
    np.testing.assert_allclose(R[:4], K @ x[:4], rtol=1e-14, atol=1e-9)
    q = net["q"]
    np.testing.assert_allclose(R[4], -(q @ K) @ x[:4], rtol=1e-13, atol=1e-9)


def test_arrhenius_temperature_scaling():
    """k(T) = A T^b exp(-E/T): ratios between two temperatures."""
    net = NETS["net7"]
    T1, T2 = np.array([1.0]), np.array([1.25])
    k1 = network.rate_constants(T1, net)[:, 0]
    k2 = network.rate_constants(T2, net)[:, 0]
    expect = (1.25 ** net["b"]) * np.exp(-net["E"] / 1.25 + net["E"] / 1.0)
    np.testing.assert_allclose(k2 / k1, expect, rtol=1e-13)
    np.testing.assert_allclose(k1, np.exp(net["lnA"] - net["E"]), rtol=1e-14)
