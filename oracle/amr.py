"""Two-level SDC with refined patches and subcycling in time (oracle; test
infrastructure only).

The paper's SDC method runs on single levels; extending it to adaptive mesh
refinement with subcycling in time is named as work under way (Sec. 2,
Sec. 5) and no algorithm is given.  Reading, a Berger-Colella-style hierarchy
around the SDC step of sdc.py:

* Levels.  Level 0 is the periodic coarse grid.  Level 1 is a set of patches,
  each a box of coarse zones refined by r = 2 in every direction, two or more
  coarse zones apart from each other and from itself across the periodic
  boundary (so every coarse zone next to a patch is uncovered), stored with
  G = 2 ghost zones per side (the stencil radius of A), x fastest.
* A coarse step of length dt:
  1. the coarse level takes one SDC step on the whole grid, covered zones
     included;
  2. every patch takes r SDC steps of dt / r.  Before every evaluation of A
     (at each node of each iteration) its ghost zones are filled from the
     coarse level: the coarse node states of the coarse step's last
     iteration, interpolated in time by the Lagrange polynomial through the
     coarse node times to the fine node's time (substep s, node m:
     theta = (s + tau_m) / r), then in space by conservative piecewise-linear
     interpolation with central coarse slopes (a fine zone at offset +-1/4
     coarse zone from its parent's centre takes U_c +- s_d / 4 per direction).
     A is set to zero in the ghost zones, whose transitions are then pure
     reaction updates that the next fill overwrites;
  3. every covered coarse zone takes the average of its 2^d fine zones, and
     every uncovered coarse zone that shares a face with a patch is refluxed:
     its update used the coarse flux through that face and takes instead the
     fine fluxes of the r substeps, averaged over the coarse face.
* The time-integrated flux an SDC step applies through a face is what its
  last sweep telescopes to:
  sum_{m=1}^{M-1} dt_m (F^{m,(K)} - F^{m,(K-1)}) + dt sum_j w_j F^{j,(K-1)},
  with w_j = sum_m S_mj the quadrature weights and F^{j,(k)} the face flux of
  node j's state at iteration k (node 0 does not change between iterations).
* Every other reading of sdc.py (nodes, quadrature, Newton, reactive source)
  applies on both levels unchanged; the second-order spatial scheme only.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass

import numpy as np

from . import advection, sdc

RATIO = 2
GHOST = 2


@dataclass
class Patch:
    lo: tuple   # first covered coarse zone, per direction (x first)
    ext: tuple  # covered coarse zones per direction (x first)


def lagrange_weights(tau, theta):
    """l_i(theta) of the Lagrange polynomials through the node times tau."""
    w = np.ones(len(tau))
    for i, ti in enumerate(tau):
        for j, tj in enumerate(tau):
            if j != i:
                w[i] *= (theta - tj) / (ti - tj)
    return w


class Hierarchy:
    """A periodic coarse grid (problem `prob`) and its refined patches."""

    def __init__(self, prob: sdc.Problem, patches):
        self.prob = prob
        self.patches = [Patch(tuple(p.lo), tuple(p.ext)) for p in patches]
        d = prob.dim
        for p in self.patches:
            if len(p.lo) != d or len(p.ext) != d:
                raise ValueError("patch corners need one entry per direction")
            for e in range(d):
                if p.ext[e] < 1 or p.lo[e] < 0 or p.lo[e] + p.ext[e] > prob.shape[e]:
                    raise ValueError("patch must lie inside the coarse grid")
                if p.ext[e] + 2 > prob.shape[e]:
                    raise ValueError("a patch must leave two coarse zones uncovered along every direction")
        for i, a in enumerate(self.patches):
            for b in self.patches[i + 1:]:
                # gaps of two or more zones on both sides of the periodic grid, along some direction
                n = prob.shape
                apart = any((a.lo[e] + a.ext[e] + 2 <= b.lo[e] and b.lo[e] + b.ext[e] + 2 <= a.lo[e] + n[e]) or
                            (b.lo[e] + b.ext[e] + 2 <= a.lo[e] and a.lo[e] + a.ext[e] + 2 <= b.lo[e] + n[e])
                            for e in range(d))
                if not apart:
                    raise ValueError("patches must be two or more coarse zones apart")

    def fine_problem(self, p: Patch):
        pc = self.prob
        shape = tuple(RATIO * e + 2 * GHOST for e in p.ext)
        return dataclasses.replace(pc, shape=shape, dx=[h / RATIO for h in pc.dx[:pc.dim]])

    # ------------------------------------------------------------ indexing
    def fine_parents(self, p: Patch, e):
        """Per padded fine index along direction e: the parent coarse zone
        (periodic) and the offset of the fine centre from the parent's centre
        (-1/4 or +1/4 coarse zone)."""
        f = np.arange(RATIO * p.ext[e] + 2 * GHOST)
        g = RATIO * p.lo[e] + (f - GHOST)      # global fine index
        par = np.floor_divide(g, RATIO)
        sigma = np.where(g - RATIO * par == 0, -0.25, 0.25)
        return np.mod(par, self.prob.shape[e]), sigma

    def ghost_mask(self, p: Patch):
        """True on the ghost zones of the padded patch array (C order)."""
        d = self.prob.dim
        inner = np.ones((), dtype=bool)
        for e in reversed(range(d)):  # C order: z, y, x
            n = RATIO * p.ext[e] + 2 * GHOST
            ok = np.zeros(n, dtype=bool)
            ok[GHOST:n - GHOST] = True
            inner = np.logical_and.outer(inner, ok) if inner.ndim else ok
        return ~inner

    def interpolate(self, Uc, p: Patch):
        """Conservative piecewise-linear values of the coarse field Uc on every
        zone of the padded patch."""
        d = self.prob.dim
        idx, sig = zip(*(self.fine_parents(p, e) for e in range(d)))
        grid_idx = np.ix_(*[idx[e] for e in reversed(range(d))])
        out = Uc[(slice(None),) + grid_idx].copy()
        for e in range(d):
            ax = Uc.ndim - 1 - e
            slope = 0.5 * (np.roll(Uc, -1, axis=ax) - np.roll(Uc, 1, axis=ax))
            shape = [1] * (d + 1)
            shape[d - e] = -1
            out = out + sig[e].reshape(shape) * slope[(slice(None),) + grid_idx]
        return out

    def average_down(self, Uf, p: Patch):
        """Mean of the 2^d fine zones of every covered coarse zone."""
        d = self.prob.dim
        inner = Uf[(slice(None),) + (slice(GHOST, -GHOST),) * d]
        acc = 0.0
        for corner in np.ndindex(*(RATIO,) * d):
            acc = acc + inner[(slice(None),) + tuple(slice(c, None, RATIO) for c in corner)]
        return acc / RATIO ** d

    def coarse_slices(self, p: Patch):
        d = self.prob.dim
        return (slice(None),) + tuple(slice(p.lo[e], p.lo[e] + p.ext[e]) for e in reversed(range(d)))


class PatchLevel:
    """The fine level of one patch during substep s: ghost fills from the
    coarse node states of the current coarse step, A zero in ghost zones."""

    def __init__(self, hier: Hierarchy, p: Patch, coarse_nodes, s):
        self.h, self.p, self.cn, self.s = hier, p, coarse_nodes, s
        self.pf = hier.fine_problem(p)
        self.tau, _ = sdc.node_times(hier.prob)
        self.mask = hier.ghost_mask(p)

    def theta(self, node):
        return (self.s + self.tau[node]) / RATIO

    def prepare(self, U, node):
        w = lagrange_weights(self.tau, self.theta(node))
        Uc_t = sum(wi * Ui for wi, Ui in zip(w, self.cn))
        fill = self.h.interpolate(Uc_t, self.p)
        out = U.copy()
        out[:, self.mask] = fill[:, self.mask]
        return out

    def A(self, U):
        A = sdc.A_of(U, self.pf)
        A[:, self.mask] = 0.0
        return A


def level_step(U, dt, prob: sdc.Problem, level=None, stats=None):
    """One SDC step of a level; returns the node states of the last two
    iterations (K-1 and K).  A(U^n) and R(U^n) are evaluated afresh (the
    synchronisation changes the state between steps)."""
    M = prob.n_nodes - 1
    U0 = level.prepare(U, 0) if level is not None else U
    A0 = level.A(U0) if level is not None else sdc.A_of(U0, prob)
    R0 = sdc.R_of_state(U0, prob)
    Uk, A, R = [U0] * (M + 1), [A0] * (M + 1), [R0] * (M + 1)
    prev = Uk
    for _ in range(prob.n_iters):
        prev = Uk
        Uk, A, R = sdc.sweep(U0, A, R, Uk, dt, prob, stats, level=level)
    return prev, Uk


def step_flux(prev, cur, dt, prob: sdc.Problem, d):
    """Time-integrated face flux along d of one SDC step (module docstring)."""
    tau, S = sdc.node_times(prob)
    M = prob.n_nodes - 1
    w = S.sum(axis=0)

    def F(U):
        if not prob.advection:  # A = 0: no flux through any face
            return np.zeros_like(U)
        return advection.face_flux(U, d, prob.dim, prob.gamma, prob.slope, prob.alpha)

    out = dt * sum(w[j] * F(prev[j]) for j in range(M + 1))
    for m in range(1, M):
        out = out + (tau[m + 1] - tau[m]) * dt * (F(cur[m]) - F(prev[m]))
    return out


def init_patches(Uc, hier: Hierarchy):
    """Patch states interpolated from the coarse state (ghosts included)."""
    return [hier.interpolate(Uc, p) for p in hier.patches]


def amr_step(Uc, Ufs, dt, hier: Hierarchy, stats=None):
    """One coarse step of the two-level hierarchy (module docstring).
    Returns the new coarse state and patch states."""
    pc = hier.prob
    d = pc.dim
    M = pc.n_nodes - 1
    prev, cur = level_step(Uc, dt, pc, None, stats)
    Uc_new = cur[M].copy()
    Fc = [step_flux(prev, cur, dt, pc, e) for e in range(d)]
    Ufs_new = []
    for p, Uf in zip(hier.patches, Ufs):
        pf = hier.fine_problem(p)
        Ff = [0.0] * d
        for s in range(RATIO):
            lvl = PatchLevel(hier, p, cur, s)
            fprev, fcur = level_step(Uf, dt / RATIO, pf, lvl, stats)
            for e in range(d):
                Ff[e] = Ff[e] + step_flux(fprev, fcur, dt / RATIO, pf, e)
            Uf = fcur[M]
        Ufs_new.append(Uf)
        reflux(Uc_new, Fc, Ff, p, hier)
        Uc_new[hier.coarse_slices(p)] = hier.average_down(Uf, p)
    return Uc_new, Ufs_new


def reflux(Uc, Fc, Ff, p: Patch, hier: Hierarchy):
    """Replace the coarse flux through the patch's faces by the averaged fine
    fluxes in the uncovered coarse zones next to them (in place)."""
    pc = hier.prob
    d = pc.dim
    for e in range(d):
        ax_c = Uc.ndim - 1 - e
        h = pc.dx[e]
        # transverse coarse range and the matching fine faces (pairs)
        for side in (0, 1):
            ci = p.lo[e] - 1 if side == 0 else p.lo[e] + p.ext[e] - 1  # coarse zone whose i+1/2 face it is
            fi = GHOST - 1 if side == 0 else GHOST + RATIO * p.ext[e] - 1  # fine zone whose i+1/2 face it is
            zone = (p.lo[e] - 1) % pc.shape[e] if side == 0 else (p.lo[e] + p.ext[e]) % pc.shape[e]
            sel_c = [slice(None)] * Uc.ndim
            sel_u = [slice(None)] * Uc.ndim
            sel_f = [slice(None)] * Uc.ndim
            for t in range(d):
                axt = Uc.ndim - 1 - t
                if t == e:
                    sel_c[axt] = ci % pc.shape[e]
                    sel_u[axt] = zone
                    sel_f[axt] = fi
                else:
                    sel_c[axt] = slice(p.lo[t], p.lo[t] + p.ext[t])
                    sel_u[axt] = slice(p.lo[t], p.lo[t] + p.ext[t])
                    sel_f[axt] = slice(GHOST, GHOST + RATIO * p.ext[t])
            fc = Fc[e][tuple(sel_c)]
            ff = Ff[e][tuple(sel_f)]
            # average the fine faces over each coarse face (pairs along every
            # transverse direction)
            for t in range(d):
                if t != e:
                    axt = ff.ndim - 1 - (t if t < e else t - 1)
                    ff = 0.5 * (np.take(ff, range(0, ff.shape[axt], 2), axis=axt)
                                + np.take(ff, range(1, ff.shape[axt], 2), axis=axt))
            corr = (ff - fc) / h
            Uc[tuple(sel_u)] += -corr if side == 0 else corr
        del ax_c


def composite_totals(Uc, Ufs, hier: Hierarchy):
    """Sums of rho, rho u_d and rho E + q . rho X over the composite grid
    (uncovered coarse zones and patch interiors), weighted by zone volume.
    Accumulated in extended precision: on grids of 10^7 zones the rounding of
    float64 sums alone reaches 1e-13 of the totals, above the conservation
    they are meant to show."""
    pc = hier.prob
    d = pc.dim
    q = np.asarray(pc.net["q"], dtype=np.longdouble)
    dVc = np.longdouble(np.prod(pc.dx[:d]))
    dVf = dVc / RATIO ** d

    def rows(U):
        Uf = U.reshape(U.shape[0], -1).astype(np.longdouble)
        return np.concatenate([Uf[:1 + d], (Uf[1 + d] + q @ Uf[2 + d:])[None]], axis=0)

    covered = np.zeros(Uc.shape[1:], dtype=bool)
    for p in hier.patches:
        covered[hier.coarse_slices(p)[1:]] = True
    tot = rows(Uc[:, ~covered]).sum(axis=1) * dVc
    for p, Uf in zip(hier.patches, Ufs):
        inner = Uf[(slice(None),) + (slice(GHOST, -GHOST),) * d]
        tot = tot + rows(inner).sum(axis=1) * dVf
    return tot
