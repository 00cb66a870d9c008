"""Pins of the oracle's fourth-order method (paper Sec. 2: Simpson's rule in
time with McCorquodale and Colella's fourth-order spatial reconstruction).

Each test measures the oracle against something its code does not contain:
exact zone averages of polynomials, Gauss-Legendre quadrature of smooth
fields (zone averages of the state, of the reactive source and of the time
derivative of an exact Euler solution), and the convergence of the whole SDC
step under refinement in space and time together.
"""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import fourth_order as fo
from oracle import sdc
from tests.test_oracle_hydro import U_INF, isentropic_vortex

GAMMA = 1.4
GL_X, GL_W = np.polynomial.legendre.leggauss(6)  # 6-point rule on [-1, 1]


def zone_average_2d(f, n):
    """Zone averages of f(X, Y) on the n x n periodic unit grid by a 6 x 6
    Gauss-Legendre rule per zone (exact to degree 11)."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    acc = 0.0
    for a, wa in zip(GL_X, GL_W):
        for b, wb in zip(GL_X, GL_W):
            Y, X = np.meshgrid(c + 0.5 * h * b, c + 0.5 * h * a, indexing="ij")
            acc = acc + 0.25 * wa * wb * f(X, Y)
    return acc


def zone_average_1d(f, n):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    return sum(0.5 * w * f(c + 0.5 * h * a) for a, w in zip(GL_X, GL_W))


def orders(errs):
    e = np.asarray(errs)
    return np.log2(e[:-1] / e[1:])


# ------------------------------------------------------------ conversions
def test_conversions_are_exact_for_cubics():
    """u_c = <u> - 1/24 Lap <u> and <f> = f_c + 1/24 Lap f_c are exact for
    polynomials of total degree <= 3 (interior zones of a non-periodic
    field): the exact zone averages of monomials are integrated by hand."""
    n, h = 12, 0.1
    x0 = 0.3 + h * np.arange(n)  # left edges
    def avg_mono(p, a):  # exact average of t^p over [a, a + h]
        return ((a + h) ** (p + 1) - a ** (p + 1)) / ((p + 1) * h)
    Y0, X0 = np.meshgrid(x0, x0, indexing="ij")
    Yc, Xc = Y0 + 0.5 * h, X0 + 0.5 * h
    terms = [((3, 0), 0.7), ((2, 1), -1.3), ((1, 2), 0.4), ((0, 3), 2.1), ((2, 0), 1.0), ((1, 1), -0.6),
             ((0, 2), 0.9), ((1, 0), 0.2), ((0, 0), 1.5)]
    avg = sum(c * avg_mono(px, X0) * avg_mono(py, Y0) for (px, py), c in terms)
    pt = sum(c * Xc ** px * Yc ** py for (px, py), c in terms)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(fo.to_centres(avg, 2)[inner], pt[inner], rtol=0, atol=1e-13)
    np.testing.assert_allclose(fo.to_averages(pt, 2)[inner], avg[inner], rtol=0, atol=1e-13)
    # a quartic term is not exact: the conversion is fourth order, not fifth
    avg4 = avg_mono(4, X0) * avg_mono(0, Y0)
    assert np.abs(fo.to_centres(avg4, 2) - Xc ** 4)[inner].max() > 1e-7


def test_face_average_is_exact_for_cubics():
    """The face interpolation 7/12 (u_i + u_{i+1}) - 1/12 (u_{i-1} + u_{i+2})
    of zone averages of a cubic equals the cubic at the face (1D)."""
    h = 0.05
    a = 0.2 + h * np.arange(20)
    f = lambda t: 1.0 - 2.0 * t + 0.5 * t ** 2 + 3.0 * t ** 3
    F = lambda t: t - t ** 2 + t ** 3 / 6 + 0.75 * t ** 4
    avg = (F(a + h) - F(a)) / h
    face = fo.face_average(avg, 0)  # at a + h
    np.testing.assert_allclose(face[1:-2], f(a + h)[1:-2], rtol=0, atol=1e-13)


def test_centre_values_converge_at_fourth_order():
    f = lambda X, Y: np.exp(np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y))
    errs = []
    for n in (16, 32, 64):
        c = (np.arange(n) + 0.5) / n
        Y, X = np.meshgrid(c, c, indexing="ij")
        errs.append(np.abs(fo.to_centres(zone_average_2d(f, n), 2) - f(X, Y)).max())
    o = orders(errs)
    assert o[-1] > 3.8, (errs, o)


# ---------------------------------------------------------------- A(U)
def vortex_dudt_average(n, R=0.1):
    """Exact zone average of dU/dt = -(U_INF . grad) U0 for the isentropic
    vortex: -U_INF,x / h times the y-face integral of the jump of U across
    the zone in x, and likewise in y (6-point Gauss-Legendre on each face)."""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    acc = 0.0
    for a, w in zip(GL_X, GL_W):
        Y, X = np.meshgrid(c + 0.5 * h * a, c, indexing="ij")  # points along y-extent, x at centres
        jx = isentropic_vortex(X + 0.5 * h, Y, R=R) - isentropic_vortex(X - 0.5 * h, Y, R=R)
        Y2, X2 = np.meshgrid(c, c + 0.5 * h * a, indexing="ij")
        jy = isentropic_vortex(X2, Y2 + 0.5 * h, R=R) - isentropic_vortex(X2, Y2 - 0.5 * h, R=R)
        acc = acc + 0.5 * w * (U_INF[0] * jx + U_INF[1] * jy)
    return -acc / h


def test_advective_term_of_the_isentropic_vortex_is_fourth_order():
    """<A(U)> of the exact zone averages of the isentropic vortex converges at
    fourth order to the exact zone average of dU/dt on every component (mass,
    momenta, energy, species).  Pressure and velocity vary, so every flux term
    and the equation of state enter; the transverse corrections of the face
    values and fluxes are needed for fourth order in 2D (without them the
    error is second order)."""
    errs, errs2 = [], []
    for n in (32, 64, 128, 256):
        Uavg = zone_average_2d(lambda X, Y: isentropic_vortex(X, Y, R=0.1), n)
        exact = vortex_dudt_average(n)
        A = fo.advective_term4(Uavg, 2, [1.0 / n, 1.0 / n], GAMMA)
        # the vortex is periodic only up to exp(-12): measure inside the
        # central 0.7 x 0.7, away from the wrapped stencils
        win = (slice(None), slice(int(0.15 * n), int(0.85 * n)), slice(int(0.15 * n), int(0.85 * n)))
        scale = np.abs(exact[win]).max(axis=(1, 2))
        errs.append(np.abs(A - exact)[win].max(axis=(1, 2)) / scale)
        # the same without the transverse corrections: second order only
        A2 = np.zeros_like(Uavg)
        for d in range(2):
            ax = 2 - d
            Ff, _, _ = fo.euler_flux(fo.face_average(Uavg, ax), d, 2, GAMMA)
            A2 -= (Ff - np.roll(Ff, 1, axis=ax)) * n
        errs2.append(np.abs(A2 - exact)[win].max(axis=(1, 2)) / scale)
    o = orders(errs)
    print("per-component errors", np.array(errs), "orders", o)
    assert np.all(o[-1] > 3.6), o
    assert np.all(np.array(errs)[-1] < 1e-4)
    o2 = orders(errs2)
    assert np.min(o2[-1]) < 2.5 and np.max(errs2[-1]) > 10 * np.max(errs[-1]), (o2, errs2[-1])


def test_uniform_state_and_conservation():
    """A uniform state gives A = 0 exactly; on a periodic grid the zone sum
    of A vanishes (fluxes telescope) to rounding."""
    w = si.workload("net2d", shape=(16, 12))
    U = w["U0"]
    Uu = np.broadcast_to(U[:, :1, :1], U.shape).copy()
    assert np.all(fo.advective_term4(Uu, 2, w["dx"], GAMMA) == 0.0)
    A = fo.advective_term4(U, 2, w["dx"], GAMMA)
    tot = np.abs(A).sum(axis=(1, 2))
    assert np.all(np.abs(A.sum(axis=(1, 2))) <= 1e-13 * tot)


# ------------------------------------------------------- reactive source
def test_average_source_is_fourth_order():
    """<R> = to_averages(R(to_centres(<U>))) converges at fourth order to the
    exact zone average of R(U(x)) (Gauss-Legendre in every zone), where R of
    the averages, R(<U>), is only second order."""
    net = si.random_network(7, 10, si.SEEDS["net7_network"])
    prob = sdc.Problem(dim=2, shape=(1, 1), dx=[1, 1], gamma=GAMMA, net=net)

    def state(X, Y):
        T = 1.0 + 0.1 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * (Y + 0.2))
        rho = 1.0 / T
        Xs = np.stack([0.9 + 0.0 * X] + [0.1 / 6 * (1 + 0.5 * np.sin(2 * np.pi * (X + s / 7.0)))
                                          for s in range(6)])
        Xs = Xs / Xs.sum(0)
        return si.conserved_from_primitive(rho, [0.1 * np.sin(2 * np.pi * Y), 0.05 + 0 * X], rho * T, Xs, GAMMA)

    def R_point(U):
        p = sdc.Problem(dim=2, shape=U.shape[1:][::-1], dx=[1, 1], gamma=GAMMA, net=net)
        return sdc.R_of_state_point(U, p)

    errs, errs2 = [], []
    for n in (16, 32, 64):
        p4 = sdc.Problem(dim=2, shape=(n, n), dx=[1 / n, 1 / n], gamma=GAMMA, net=net, space_order=4)
        Uavg = zone_average_2d(state, n)
        exact = zone_average_2d(lambda X, Y: R_point(state(X, Y)), n)
        scale = np.abs(exact).max()
        errs.append(np.abs(sdc.R_of_state(Uavg, p4) - exact).max() / scale)
        errs2.append(np.abs(R_point(Uavg) - exact).max() / scale)
    assert orders(errs)[-1] > 3.7, errs
    assert orders(errs2)[-1] < 2.3, errs2
    del prob


# ------------------------------------------------------------ the method
def smooth_reacting_1d(n, rates):
    """Exact zone averages of a smooth 1D reacting flow: density, velocity and
    pressure waves and a species profile, with a non-stiff linear chain."""
    def U(x):
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
        u = 0.3 + 0.1 * np.sin(2 * np.pi * x + 1.0)
        p = 1.0 + 0.1 * np.cos(2 * np.pi * x)
        a = 0.6 + 0.2 * np.sin(2 * np.pi * x + 0.5)
        X = np.stack([a, 0.8 - a, 0.1 + 0 * x, 0.1 + 0 * x])
        return si.conserved_from_primitive(rho, [u], p, X, GAMMA)
    return zone_average_1d(U, n), si.chain_network(rates=rates)


def restrict(U):
    """Zone averages on the grid one level coarser (pairs of zones)."""
    return 0.5 * (U[..., 0::2] + U[..., 1::2])


@pytest.mark.parametrize("space_order,n_nodes,n_iters,expect", [(4, 3, 4, (3.6, 5.0)), (2, 3, 4, (1.5, 2.5))])
def test_method_converges_at_fourth_order_in_space_and_time(space_order, n_nodes, n_iters, expect):
    """The whole SDC step with dt proportional to h: with the fourth-order
    advective term and zone-average sources (Simpson, K = 4) the solution
    converges at fourth order in space and time together; with the
    second-order spatial scheme (smooth mode) the same run is second order.
    Errors against the next finer run averaged onto the coarse zones."""
    T = 0.1
    sols = []
    for n in (32, 64, 128, 256):
        U0, net = smooth_reacting_1d(n, rates=(3.0, 2.0, 1.0))
        p = sdc.Problem(dim=1, shape=(n,), dx=[1.0 / n], gamma=GAMMA, net=net, n_nodes=n_nodes,
                        n_iters=n_iters, slope=0, alpha=2.0, space_order=space_order)
        nsteps = n // 4  # (|u| + c) dt / h = 0.64
        sols.append(sdc.run(U0, T / nsteps, nsteps, p))
    errs = [np.abs(restrict(sols[i + 1]) - sols[i]).max(axis=1) / np.abs(sols[i]).max(axis=1)
            for i in range(len(sols) - 1)]
    e = np.max(np.array(errs), axis=1)
    o = orders(e)
    print(f"space order {space_order}: errors {e}, orders {o}")
    assert expect[0] < o[-1] < expect[1], o
