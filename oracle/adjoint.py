"""Gradient of the integrated energy release by complex step (oracle).

The objective (a reading; the benchmark asks for the gradient of total
integrated energy release with respect to rate parameters) is

  J_E = dV sum_z sum_i q_i [rho X_i(t_0) - rho X_i(t_N)],

the total energy the reactions added to rho E (advection telescopes on the
periodic grid and R_e = -sum_i q_i R_i).  Its derivative with respect to one
rate parameter theta (lnA_r or E_r) is Im J_E(theta + i h) / h, computed by
running the whole oracle in complex arithmetic.  This needs the smooth mode
(central slopes, frozen Rusanov speed), since limiters are not analytic; the
Newton stopping test uses real parts and one extra iteration after
convergence settles the imaginary part.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import sdc


def energy_gradient(U0, dt, nsteps, prob: sdc.Problem, which="both", h=1e-30, reactions=None):
    """dJ_E/dlnA_r and dJ_E/dE_r for r in `reactions` (default all)."""
    if prob.slope != 0 or not prob.alpha > 0:
        raise ValueError("complex-step gradient needs slope=0 and a frozen alpha > 0")
    net = prob.net
    reactions = range(net["nreact"]) if reactions is None else reactions
    lnA0 = np.asarray(net["lnA"], dtype=complex)
    E0 = np.asarray(net["E"], dtype=complex)
    g_lnA, g_E = [], []
    for r in reactions:
        for kind in ("lnA", "E"):
            if which not in ("both", kind):
                continue
            lnA, E = lnA0.copy(), E0.copy()
            (lnA if kind == "lnA" else E)[r] += 1j * h
            p = dataclasses.replace(prob, lnA=lnA, E=E, newton_extra=1)
            UN = sdc.run(U0.astype(complex), dt, nsteps, p)
            J = sdc.energy_released(U0, UN, p)
            (g_lnA if kind == "lnA" else g_E).append(J.imag / h)
    return np.array(g_lnA), np.array(g_E)
