"""Pin P9: the oracle's complex-step gradient of the energy release against
central finite differences of the oracle itself."""
import dataclasses

import numpy as np

import sdc_inputs as si
from oracle import adjoint, sdc


def test_complex_step_gradient_matches_central_differences():
    w = si.workload("adjoint2d", shape=(8, 8))
    p = sdc.Problem.from_workload(w)
    nsteps = 3
    reactions = [0, 1, 4]
    g_lnA, g_E = adjoint.energy_gradient(w["U0"], w["dt"], nsteps, p, reactions=reactions)
    net = p.net

    def J(lnA, E):
        pp = dataclasses.replace(p, lnA=lnA, E=E)
        return sdc.energy_released(w["U0"], sdc.run(w["U0"], w["dt"], nsteps, pp), pp)

    fd_lnA, fd_E = [], []
    for r in reactions:
        h = 1e-4
        a, b = net["lnA"].copy(), net["lnA"].copy()
        a[r] += h
        b[r] -= h
        fd_lnA.append((J(a, net["E"]) - J(b, net["E"])) / (2 * h))
        hE = 1e-4 * net["E"][r]
        a, b = net["E"].copy(), net["E"].copy()
        a[r] += hE
        b[r] -= hE
        fd_E.append((J(net["lnA"], a) - J(net["lnA"], b)) / (2 * hE))
    for g, fd in ((g_lnA, np.array(fd_lnA)), (g_E, np.array(fd_E))):
        tol = 1e-6 * (np.abs(fd) + np.abs(fd).max())
        assert np.all(np.abs(g - fd) <= tol), (g, fd)
        assert np.abs(fd).max() > 1e-8
