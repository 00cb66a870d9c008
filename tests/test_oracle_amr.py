"""Pins of the oracle's two-level SDC with refined patches and subcycling
(the AMR extension the paper names in Sec. 2 and Sec. 5).

Each test measures the hierarchy against a fact that its code does not
contain: exact space-time interpolation of fields that are linear in space and
polynomial in time, conservation of mass, momentum and total energy on the
composite grid (which the refluxing exists for), the subcycled fine steps of a
reaction-only problem against plain single-grid steps of half the length, a
uniform state staying uniform, and second-order convergence towards a
uniformly fine run.
"""
import dataclasses

import numpy as np
import pytest

import sdc_inputs as si
from oracle import amr, sdc

GAMMA = 1.4


def problem(shape, dx, net, **over):
    kw = dict(dim=len(shape), shape=tuple(shape), dx=list(dx), gamma=GAMMA, net=net, n_nodes=3, n_iters=4,
              slope=0, alpha=2.0)
    kw.update(over)
    return sdc.Problem(**kw)


def smooth_state(shape, ns, seed=3, amp=0.1):
    """Smooth periodic primitive fields on the unit box (zone centres)."""
    g = si.rng(seed)
    dim = len(shape)
    c = [(np.arange(n) + 0.5) / n for n in shape]
    X = np.meshgrid(*c[::-1], indexing="ij")[::-1]  # X[0] = x, C order arrays
    ph = g.uniform(0, 1, size=8)
    T = 1.0 + amp * np.prod([np.sin(2 * np.pi * (X[e] + ph[e])) for e in range(dim)], axis=0) + 0 * X[0]
    rho = 1.0 / T
    u = [0.2 * np.sin(2 * np.pi * (X[(e + 1) % dim] + ph[3 + e])) + 0.1 for e in range(dim)]
    Xs = np.stack([0.7 + 0.1 * np.sin(2 * np.pi * (X[0] + ph[6]))] + [0.3 / (ns - 1) + 0 * X[0]] * (ns - 1))
    Xs[1] = 1.0 - Xs[0] - Xs[2:].sum(0)
    return si.conserved_from_primitive(rho, u, rho * T, Xs, GAMMA)


def test_ghost_fill_is_exact_for_linear_space_and_quadratic_time():
    """Coarse node states a + b x + (c + e x) t + f t^2 (linear in space per
    time, quadratic in time through 3 nodes): every fine ghost zone of every
    substep and node receives the field at its centre and its node time."""
    net = si.chain_network()
    n = 16
    pc = problem((n, n), (1 / n, 1 / n), net)
    hier = amr.Hierarchy(pc, [amr.Patch((5, 6), (4, 3))])
    p = hier.patches[0]
    tau, _ = sdc.node_times(pc)

    def field(x, y, t):
        return np.stack([1.0 + 0.3 * x - 0.2 * y + (0.5 + 0.1 * x) * t + 0.7 * t * t,
                         -0.4 + 0.05 * y + 2.0 * t])

    # coarse node states at zone centres (only the patch's neighbourhood is
    # used, away from the periodic wrap)
    cx = (np.arange(n) + 0.5) / n
    Yc, Xc = np.meshgrid(cx, cx, indexing="ij")
    nodes = [field(Xc, Yc, t) for t in tau]

    class Lvl(amr.PatchLevel):
        def __init__(self, s):
            self.h, self.p, self.cn, self.s = hier, p, nodes, s
            self.tau = tau
            self.mask = hier.ghost_mask(p)

    fx = (amr.RATIO * p.lo[0] + np.arange(amr.RATIO * p.ext[0] + 2 * amr.GHOST) - amr.GHOST + 0.5) / (2 * n)
    fy = (amr.RATIO * p.lo[1] + np.arange(amr.RATIO * p.ext[1] + 2 * amr.GHOST) - amr.GHOST + 0.5) / (2 * n)
    Yf, Xf = np.meshgrid(fy, fx, indexing="ij")
    for s in range(amr.RATIO):
        lvl = Lvl(s)
        for node in range(len(tau)):
            out = lvl.prepare(np.zeros((2,) + Xf.shape), node)
            exact = field(Xf, Yf, (s + tau[node]) / amr.RATIO)
            assert np.abs(out[:, lvl.mask] - exact[:, lvl.mask]).max() < 1e-14
            assert np.all(out[:, ~lvl.mask] == 0.0)


def test_uniform_state_stays_uniform():
    net = dict(si.chain_network(), lnA=np.full(3, -700.0))  # no reactions
    n = 12
    pc = problem((n, n), (1 / n, 1 / n), net)
    U = si.conserved_from_primitive(np.full((n, n), 1.3), [np.full((n, n), 0.2), np.full((n, n), -0.1)],
                                    np.full((n, n), 0.9), np.stack([np.full((n, n), 0.25)] * 4), GAMMA)
    hier = amr.Hierarchy(pc, [amr.Patch((2, 3), (4, 5))])
    Uc, Ufs = U, amr.init_patches(U, hier)
    for _ in range(2):
        Uc, Ufs = amr.amr_step(Uc, Ufs, 0.01, hier)
    ref = U[:, :1, :1]
    assert np.abs(Uc - ref).max() <= 1e-15 * np.abs(ref).max()
    assert np.abs(Ufs[0] - ref).max() <= 1e-15 * np.abs(ref).max()


@pytest.mark.parametrize("dim", [1, 2])
def test_composite_grid_conserves_mass_momentum_and_energy(dim):
    """Reacting smooth flow with two patches: the composite-grid totals of rho,
    rho u and rho E + q . rho X are constant to rounding; without the
    refluxing they drift at the level of the coarse/fine flux mismatch."""
    net = si.random_network(7, 10, si.SEEDS["net7_network"])
    shape = (32,) if dim == 1 else (24, 20)
    patches = [amr.Patch((4,), (6,)), amr.Patch((20,), (5,))] if dim == 1 else \
        [amr.Patch((3, 2), (6, 5)), amr.Patch((13, 11), (7, 6))]
    pc = problem(shape, [1.0 / s for s in shape], net, slope=1, alpha=-1.0)
    U = smooth_state(shape, 7)
    hier = amr.Hierarchy(pc, patches)
    dt = 0.3 * min(pc.dx) / 1.5
    Uc, Ufs = U, amr.init_patches(U, hier)
    tot0 = amr.composite_totals(Uc, Ufs, hier)
    scale = np.abs(tot0) + 1e-3
    for _ in range(3):
        Uc, Ufs = amr.amr_step(Uc, Ufs, dt, hier)
    drift = np.abs(amr.composite_totals(Uc, Ufs, hier) - tot0) / scale
    print("conservation drift", drift)
    assert np.all(drift <= 1e-15), drift
    # the same without refluxing is not conservative
    saved = amr.reflux
    try:
        amr.reflux = lambda *a, **k: None
        Uc2, Ufs2 = U, amr.init_patches(U, hier)
        for _ in range(3):
            Uc2, Ufs2 = amr.amr_step(Uc2, Ufs2, dt, hier)
    finally:
        amr.reflux = saved
    assert np.max(np.abs(amr.composite_totals(Uc2, Ufs2, hier) - tot0) / scale) > 1e-9


def test_reaction_only_subcycling():
    """With A = 0 the levels decouple: uncovered coarse zones take one coarse
    step, patch interiors two plain steps of dt / 2 on their own data, and
    covered coarse zones the average of their fine zones."""
    net = si.random_network(7, 10, si.SEEDS["net7_network"])
    shape = (10, 8)
    pc = problem(shape, [0.1, 0.125], net, advection=0)
    U = smooth_state(shape, 7)
    hier = amr.Hierarchy(pc, [amr.Patch((2, 1), (4, 3))])
    Uf0 = amr.init_patches(U, hier)
    dt = 3e-3
    Uc, Ufs = amr.amr_step(U, Uf0, dt, hier)
    ref_c = sdc.run(U, dt, 1, pc)
    pf = hier.fine_problem(hier.patches[0])
    ref_f = sdc.run(Uf0[0], dt / 2, 2, pf)
    inner = (slice(None), slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(Ufs[0][inner], ref_f[inner], rtol=1e-14, atol=0)
    covered = np.zeros(shape[::-1], dtype=bool)
    covered[hier.coarse_slices(hier.patches[0])[1:]] = True
    np.testing.assert_allclose(Uc[:, ~covered], ref_c[:, ~covered], rtol=1e-14, atol=0)
    np.testing.assert_allclose(Uc[hier.coarse_slices(hier.patches[0])],
                               hier.average_down(ref_f, hier.patches[0]), rtol=1e-14, atol=0)


def test_two_level_run_converges_to_the_uniformly_fine_run():
    """1D smooth reacting flow, patch over the middle half: the patch zones
    approach the uniformly fine run of the same method at second order as the
    grids are refined together, and the uncovered coarse zones stay as close
    to it (averaged) as a plain coarse run does."""
    net = si.chain_network(rates=(3.0, 2.0, 1.0))
    T = 0.1
    e_fine, e_coarse, e_plain = [], [], []
    for n in (32, 64, 128, 256):
        pc = problem((n,), (1.0 / n,), net)
        pf_uni = problem((2 * n,), (0.5 / n,), net)
        Uf_uni = smooth_state((2 * n,), 4)
        Uc = 0.5 * (Uf_uni[:, 0::2] + Uf_uni[:, 1::2])
        Uc0 = Uc.copy()
        hier = amr.Hierarchy(pc, [amr.Patch((n // 4,), (n // 2,))])
        # patch initial data: the uniform fine data on its zones (ghosts too)
        Ufs = [Uf_uni[:, (n // 2 - amr.GHOST):(n // 2 + n + amr.GHOST)].copy()]
        nsteps = n // 4
        dt = T / nsteps  # (|u| + c) dt / h about 0.3 on both levels
        for _ in range(nsteps):
            Uc, Ufs = amr.amr_step(Uc, Ufs, dt, hier)
        ref = sdc.run(Uf_uni, dt / 2, 2 * nsteps, pf_uni)
        ref_c = 0.5 * (ref[:, 0::2] + ref[:, 1::2])
        unc = np.r_[0:n // 4, 3 * n // 4:n]
        e_fine.append(np.abs(Ufs[0][:, amr.GHOST:-amr.GHOST] - ref[:, n // 2:n // 2 + n]).max())
        e_coarse.append(np.abs(Uc[:, unc] - ref_c[:, unc]).max())
        e_plain.append(np.abs(sdc.run(Uc0, dt, nsteps, pc)[:, unc] - ref_c[:, unc]).max())
    o = np.log2(np.array(e_fine[:-1]) / np.array(e_fine[1:]))
    print("patch errors", e_fine, "orders", o, "uncovered", e_coarse, "plain coarse", e_plain)
    assert o[-1] > 1.9, (e_fine, o)
    assert np.all(np.array(e_coarse) <= 1.2 * np.array(e_plain))


def test_patches_meeting_across_the_periodic_boundary_are_rejected():
    """Patches two zones apart inside the grid but touching through the
    periodic boundary, and a patch that meets itself through it, would make
    a covered coarse zone the reflux target of an interface face."""
    net = si.chain_network()
    pc = problem((16, 12), (1 / 16, 1 / 12), net)
    amr.Hierarchy(pc, [amr.Patch((2, 2), (4, 4)), amr.Patch((8, 2), (6, 4))])  # 2 zones apart both ways
    with pytest.raises(ValueError, match="apart"):
        amr.Hierarchy(pc, [amr.Patch((1, 2), (4, 4)), amr.Patch((8, 2), (8, 4))])  # one zone apart across x = 0
    with pytest.raises(ValueError, match="uncovered"):
        amr.Hierarchy(pc, [amr.Patch((0, 2), (15, 4))])
