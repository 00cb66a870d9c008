"""Pins of the oracle's hydrodynamics: the Euler flux and equation of state
inside A(U) (paper Sec. 2, Eq. 1: A is the divergence of the hydro fluxes) and
the energy objective of the adjoint.

Each test checks the oracle against a fact of gas dynamics that is fixed
independently of its code: an exact moving solution of the Euler equations,
the eigenvalues of the flux Jacobian, the normal-shock jump conditions and
the volume integral of the energy the reactions release.
"""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import advection, eos, sdc

GAMMA = 1.4
U_INF = (0.7, 0.4)


def isentropic_vortex(X, Y, R=0.08, beta=5.0, ns=3, gamma=GAMMA):
    """Conserved state of the isentropic vortex (Shu's test problem) centred
    at (1/2, 1/2) with radius scale R, on the free stream U_INF, plus passive
    species whose mass fractions depend on the radius only.  The vortex is an
    exact solution of the Euler equations that moves rigidly with the free
    stream, U(x, t) = U0(x - U_INF t), and a mass fraction constant on the
    vortex's circular streamlines is carried along with it, so
    dU/dt = A(U) = -(U_INF . grad) U0.  Accepts complex coordinates (complex
    step differentiation)."""
    xb, yb = (X - 0.5) / R, (Y - 0.5) / R
    r2 = xb * xb + yb * yb
    f = np.exp(0.5 * (1.0 - r2))
    du = -beta / (2 * np.pi) * f * yb
    dv = beta / (2 * np.pi) * f * xb
    T = 1.0 - (gamma - 1.0) * beta ** 2 / (8 * gamma * np.pi ** 2) * f * f
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T  # isentropic: p = rho^gamma
    w = np.stack([1.0 + 0.5 * np.exp(-r2 * (s + 1) / 3.0) for s in range(ns)])
    return si.conserved_from_primitive(rho, [U_INF[0] + du, U_INF[1] + dv], p, w / w.sum(0), gamma)


def _vortex_errors(n, slope, alpha, norm):
    c = (np.arange(n) + 0.5) / n
    Y, X = np.meshgrid(c, c, indexing="ij")
    A = advection.advective_term(isentropic_vortex(X, Y), 2, [1 / n, 1 / n], GAMMA, slope, alpha)
    h = 1e-30  # complex step: exact derivatives of the analytic field
    exact = -(U_INF[0] * isentropic_vortex(X + 1j * h, Y).imag + U_INF[1] * isentropic_vortex(X, Y + 1j * h).imag) / h
    red = (lambda a: np.abs(a).max(axis=(1, 2))) if norm == "max" else (lambda a: np.abs(a).mean(axis=(1, 2)))
    return red(A - exact) / red(exact)


@pytest.mark.parametrize("slope,alpha,norm,order,bound", [(0, 2.5, "max", 2.0, 5e-3), (0, -1.0, "max", 2.0, 5e-3),
                                                          (1, -1.0, "l1", 1.8, 2e-2)])
def test_isentropic_vortex_is_transported(slope, alpha, norm, order, bound):
    """A(U) of the isentropic vortex converges at second order to
    -(U_INF . grad) U on every component: mass, both momenta, total energy and
    species.  Pressure and velocity vary across the vortex, so every pressure
    term of the flux and the equation of state enter (a dropped p in the
    momentum or energy flux, or p from gamma instead of gamma - 1, leaves an
    O(1) error)."""
    e = np.array([_vortex_errors(n, slope, alpha, norm) for n in (64, 128, 256)])
    rates = np.log2(e[:-1] / e[1:])
    print("errors", e[-1], "rates", rates[-1])
    assert np.all(rates[-1] > order), rates
    assert np.all(e[-1] < bound), e[-1]


def _complex_step_jacobian(U, d, dim, gamma):
    """dF_d/dU of the oracle's physical flux at one state U [n], by complex step."""
    n = U.size
    J = np.empty((n, n))
    h = 1e-30
    for j in range(n):
        V = U.astype(complex)
        V[j] += 1j * h
        F, _, _ = advection.euler_flux(V[:, None], d, dim, gamma)
        J[:, j] = F[:, 0].imag / h
    return J


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_flux_jacobian_eigenvalues_are_u_and_u_plus_minus_c(dim):
    """The eigenvalues of the Euler flux Jacobian along d are u_d - c,
    u_d (every other wave) and u_d + c, with c the sound speed: this fixes
    eos.sound_speed (the local Rusanov speed is max |u_d| + c) from the flux
    alone."""
    g = si.rng(11)
    ns = 2
    for _ in range(5):
        rho = g.uniform(0.3, 3.0, 1)
        u = [g.uniform(-2, 2, 1) for _ in range(dim)]
        p = g.uniform(0.2, 5.0, 1)
        Xs = g.uniform(0.1, 1.0, (ns, 1))
        Xs /= Xs.sum(0)
        U = si.conserved_from_primitive(rho, u, p, Xs)[:, 0]
        for d in range(dim):
            lam = np.sort(np.linalg.eigvals(_complex_step_jacobian(U, d, dim, GAMMA)).real)
            c = eos.sound_speed(U[0], eos.pressure(U[:, None], dim, GAMMA)[0], GAMMA)
            ud = U[1 + d] / U[0]
            expect = np.sort(np.concatenate([[ud - c, ud + c], np.full(U.size - 2, ud)]))
            assert np.allclose(lam, expect, rtol=0, atol=1e-9 * (abs(ud) + c)), (lam, expect)


def normal_shock(M1, rho1=1.0, p1=1.0, gamma=GAMMA):
    """Upstream and downstream primitive states (rho, u, p) of a stationary
    normal shock with upstream Mach number M1 (the textbook jump relations)."""
    u1 = M1 * np.sqrt(gamma * p1 / rho1)
    r = (gamma + 1) * M1 ** 2 / ((gamma - 1) * M1 ** 2 + 2)
    p2 = p1 * (1 + 2 * gamma / (gamma + 1) * (M1 ** 2 - 1))
    return (rho1, u1, p1), (rho1 * r, u1 / r, p2)


@pytest.mark.parametrize("M1", [1.2, 2.0, 5.0])
def test_stationary_shock_has_equal_fluxes(M1):
    """Rankine-Hugoniot: across a stationary normal shock the Euler flux is
    continuous, F(U_L) = F(U_R), for the momentum and energy components as
    well as mass and species; a tangential velocity rides along unchanged."""
    (r1, u1, p1), (r2, u2, p2) = normal_shock(M1)
    Xs = np.array([[0.3], [0.7]])
    for dim, d in ((1, 0), (2, 0), (2, 1), (3, 2)):
        def state(r, un, p):
            u = [np.full(1, 0.37 if e != d else un) for e in range(dim)]
            return si.conserved_from_primitive(np.full(1, r), u, np.full(1, p), Xs)
        UL, UR = state(r1, u1, p1), state(r2, u2, p2)
        FL, _, _ = advection.euler_flux(UL, d, dim, GAMMA)
        FR, _, _ = advection.euler_flux(UR, d, dim, GAMMA)
        scale = np.abs(FL).max()
        assert np.max(np.abs(FL - FR)) <= 1e-14 * scale, (FL[:, 0], FR[:, 0])
        # and the states do differ: this is a real jump
        assert np.max(np.abs(UL - UR)) > 0.1


def test_local_rusanov_speed_at_a_jump():
    """A state with one jump: MC slopes vanish next to it, so the face states
    are the two cell values and A in the two cells beside the jump is the
    difference between the Rusanov flux, whose speed is the largest flux-
    Jacobian eigenvalue magnitude of the two states (computed here from the
    eigenvalues, not from a sound-speed formula), and the physical flux."""
    n = 16
    rho = np.where(np.arange(n) < n // 2, 1.0, 0.4)
    u = np.where(np.arange(n) < n // 2, 0.3, -0.5)
    p = np.where(np.arange(n) < n // 2, 1.0, 2.5)
    Xs = np.stack([np.where(np.arange(n) < n // 2, 0.2, 0.9)])
    Xs = np.concatenate([Xs, 1 - Xs])
    U = si.conserved_from_primitive(rho, [u], p, Xs)
    dx = 1.0 / n
    A = advection.advective_term(U, 1, [dx], GAMMA, slope=1, alpha=-1.0)
    i = n // 2 - 1  # the jump is the face between i and i + 1
    UL, UR = U[:, i], U[:, i + 1]
    lam = max(np.abs(np.linalg.eigvals(_complex_step_jacobian(V, 0, 1, GAMMA))).max() for V in (UL, UR))
    FL, _, _ = advection.euler_flux(UL[:, None], 0, 1, GAMMA)
    FR, _, _ = advection.euler_flux(UR[:, None], 0, 1, GAMMA)
    Fj = 0.5 * (FL[:, 0] + FR[:, 0]) - 0.5 * lam * (UR - UL)
    # every other face of cells i and i + 1 joins equal states: flux = F(U)
    expect_i = -(Fj - FL[:, 0]) / dx
    expect_ip = -(FR[:, 0] - Fj) / dx
    sc = np.abs(expect_i).max()
    assert np.max(np.abs(A[:, i] - expect_i)) < 1e-13 * sc
    assert np.max(np.abs(A[:, i + 1] - expect_ip)) < 1e-13 * sc
    # the periodic wrap puts the other jump at the face between n - 1 and 0;
    # away from both jumps the state is uniform and A vanishes
    assert np.all(A[:, 3:i - 1] == 0.0)


@pytest.mark.parametrize("advect", [0, 1])
def test_energy_released_is_the_volume_integral_of_energy_gained(advect):
    """J_E is the reaction energy added to the gas over the domain: with
    periodic advection (which moves energy around but creates none) or none,
    it equals the domain volume times the mean gain of total energy density,
    on a grid whose zones are not unit cubes."""
    w = si.workload("net2d", shape=(12, 8))
    L = (0.6, 0.25)
    dx = [L[0] / 12, L[1] / 8]
    prob = sdc.Problem.from_workload(w, dx=dx, advection=advect, slope=0, alpha=2.0)
    U0 = w["U0"]
    UN = sdc.run(U0, 0.5 * w["dt"], 2, prob)
    d = prob.dim
    gained = (L[0] * L[1]) * np.mean(UN[1 + d] - U0[1 + d])
    J = sdc.energy_released(U0, UN, prob)
    assert abs(gained) > 1e-6
    assert abs(J - gained) <= 1e-12 * abs(gained), (J, gained)
