"""Synthetic reaction network: rates, source R and analytic Jacobian (oracle).

The paper's reactive source R(U) (Sec. 2, Eq. 1) acts only on the partial
densities and the energy; mass and momentum have no reactive source.  The
network itself is synthetic (no physical rate data).  Reading of its rate law:

  x      = (rho X_1, ..., rho X_Ns, rho e)      reacting variables
  T      = (gamma - 1) x_e / rho                (gamma-law, p = rho T)
  k_r    = exp(lnA_r + b_r ln T - E_r / T)      Arrhenius / power law
  v_r    = k_r * x_a            (unimolecular, reactant a)
         = k_r * x_a * x_c      (bimolecular, reactants a and c)
           v_r is rho times the molar-free rate w_r of the mass-fraction form
  R_i    = sum_r s_ir v_r                       species source (sum_i s_ir = 0)
  R_e    = sum_r Q_r v_r,  Q_r = -sum_i s_ir q_i   energy released

so that R_e = -sum_i q_i R_i for every evaluation (energy conservation).

All functions accept complex arrays, so complex-step derivatives pass through.
"""
from __future__ import annotations

import numpy as np


def q_values(net):
    """Q_r = -sum_i s_ir q_i (energy released per unit reaction rate)."""
    return -(net["stoich"] @ net["q"])


def rate_constants(T, net, lnA=None, E=None):
    """k_r(T) for every reaction, shape [nreact, Z]."""
    lnA = net["lnA"] if lnA is None else lnA
    E = net["E"] if E is None else E
    lnT = np.log(T)
    return np.exp(lnA[:, None] + net["b"][:, None] * lnT[None] - E[:, None] / T[None])


def monomials(x, net):
    """Reactant products m_r (v_r = k_r m_r) and their partial derivatives.

    Returns m [nreact, Z] and a list of (reactant index, dm/dx_reactant) pairs
    per reaction.
    """
    nr = net["nreact"]
    Z = x.shape[1]
    m = np.empty((nr, Z), dtype=x.dtype)
    dm = []
    for r in range(nr):
        a, c = (int(v) for v in net["reactants"][r])
        if c < 0:
            m[r] = x[a]
            dm.append([(a, np.ones(Z, dtype=x.dtype))])
        else:
            m[r] = x[a] * x[c]
            dm.append([(a, x[c]), (c, x[a])])
    return m, dm


def source(x, rho, net, gamma, lnA=None, E=None):
    """R(x; rho) on the reacting variables, shape [Ns+1, Z]."""
    ns = net["nspec"]
    T = (gamma - 1.0) * x[ns] / rho
    k = rate_constants(T, net, lnA, E)
    m, _ = monomials(x, net)
    v = k * m
    R = np.empty_like(x, dtype=np.result_type(x, v))
    R[:ns] = net["stoich"].T @ v
    R[ns] = q_values(net) @ v
    return R


def source_and_jacobian(x, rho, net, gamma, lnA=None, E=None):
    """R(x; rho) [n, Z] and the analytic Jacobian dR/dx [Z, n, n], n = Ns+1.

    dv_r/dx_a = k_r dm_r/dx_a for each reactant a, and
    dv_r/dx_e = v_r (b_r / T + E_r / T^2) (gamma - 1) / rho.
    """
    ns = net["nspec"]
    n = ns + 1
    Z = x.shape[1]
    E_ = net["E"] if E is None else E
    T = (gamma - 1.0) * x[ns] / rho
    k = rate_constants(T, net, lnA, E)
    m, dm = monomials(x, net)
    v = k * m
    dtype = np.result_type(x, v)
    R = np.empty((n, Z), dtype=dtype)
    R[:ns] = net["stoich"].T @ v
    Q = q_values(net)
    R[ns] = Q @ v
    # rows: species i (via s_ir) and energy (via Q_r); columns: the variables
    # the rate v_r depends on.
    coeff = np.concatenate([net["stoich"], Q[:, None]], axis=1)  # [nr, n]
    J = np.zeros((Z, n, n), dtype=dtype)
    dTdxe = (gamma - 1.0) / rho
    for r in range(net["nreact"]):
        for a, dma in dm[r]:
            J[:, :, a] += (k[r] * dma)[:, None] * coeff[r][None, :]
        dv_e = v[r] * (net["b"][r] / T + E_[r] / (T * T)) * dTdxe
        J[:, :, ns] += dv_e[:, None] * coeff[r][None, :]
    return R, J


def source_param_derivatives(x, rho, net, gamma):
    """dR/dlnA_r and dR/dE_r at fixed x, each [nreact, n, Z].

    dv_r/dlnA_r = v_r and dv_r/dE_r = -v_r / T.
    """
    ns = net["nspec"]
    T = (gamma - 1.0) * x[ns] / rho
    k = rate_constants(T, net)
    m, _ = monomials(x, net)
    v = k * m
    coeff = np.concatenate([net["stoich"], q_values(net)[:, None]], axis=1)
    dlnA = coeff[:, :, None] * v[:, None, :]
    dE = -coeff[:, :, None] * (v / T[None])[:, None, :]
    return dlnA, dE


def source_full(U, dim, net, gamma):
    """R(U) on the full conserved vector (zeros on rho and rho u).

    The reacting variables are x = (rho X, rho E - 0.5|rho u|^2/rho).
    """
    ns = net["nspec"]
    shape = U.shape[1:]
    Uf = U.reshape(U.shape[0], -1)
    rho = Uf[0]
    ke = 0.0
    for d in range(dim):
        ke = ke + Uf[1 + d] * Uf[1 + d]
    ke = 0.5 * ke / rho
    x = np.concatenate([Uf[2 + dim:2 + dim + ns], (Uf[1 + dim] - ke)[None]], axis=0)
    R = source(x, rho, net, gamma)
    out = np.zeros_like(Uf, dtype=R.dtype)
    out[1 + dim] = R[ns]
    out[2 + dim:] = R[:ns]
    return out.reshape((U.shape[0],) + shape)
