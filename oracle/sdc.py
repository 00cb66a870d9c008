"""SDC correction sweep, per-zone Newton reaction solve and time step (oracle).

Follows Sec. 2, Eq. 2 of the paper: the update from node m to m+1 at
iteration k+1 is

  U^{m+1,(k+1)} = U^{m,(k+1)} + dt_m [A^{m,(k+1)} - A^{m,(k)}]
                + dt_m [R^{m+1,(k+1)} - R^{m+1,(k)}]
                + int_{t^m}^{t^{m+1}} (A^{(k)} + R^{(k)}) dt,

an implicit equation for U^{m+1,(k+1)} because R^{m+1,(k+1)} = R(U^{m+1,(k+1)}).
The integral uses the previous iteration's values at all nodes through the
matrix S of `quadrature.py`.

Readings where the paper is silent:

* initial iterate: every node of iteration 0 holds U^n, A(U^n), R(U^n), so
  the first sweep is IMEX Euler between nodes;
* node 0 is U^n at every iteration, so A^{0,(k+1)} - A^{0,(k)} = 0;
* the step ends with U^{n+1} = U^{M,(K)} (no extra quadrature update);
* the implicit unknowns are x = (rho X, rho e): rho and rho u have no reactive
  source and are final after the explicit part, and rho E = rho e + KE with
  KE taken from the new rho and rho u;
* Newton starts from the reacting vector of U^{m+1,(k)} (the same node at the
  previous iteration), re-forms the analytic Jacobian every iteration, solves
  with LU and partial pivoting (LAPACK via numpy.linalg.solve), and measures
  each step by e_k = max_i |delta_i| / s_i with s = rho for species and |b_e|
  for the energy.  It stops after step k when e_k <= tol, or when the steps
  contract (e_k < e_{k-1}) and the contraction bounds the new iterate's
  distance from the root by tol: theta = e_k / e_{k-1}, and the distance is at
  most theta / (1 - theta) e_k = e_k^2 / (e_{k-1} - e_k) <= tol (the stopping
  test of Hairer and Wanner, Solving ODEs II, Sec. IV.8, with kappa = 1).  At
  least one iteration, at most maxiter, no damping or clipping; a zone that
  does not converge keeps its last iterate and reports -1;
* R^{m+1,(k+1)} is R re-evaluated at the converged x;
* A^0 and R^0 of step n+1 are A^{M,(K)} and R^{M,(K)} of step n (the same
  state; `run` carries them over).

Fourth order in space (space_order = 4, the paper's fourth-order method with
Simpson's rule in time; pieces in `fourth_order.py`): A is the fourth-order
zone-average advective term, and the reactive terms are zone averages of the
source at zone-centre states.  Reading of the implicit part: the right-hand
side of Eq. 2 (zone averages) is converted to zone-centre values, the Newton
solve runs on those (same guess, stopping rule and unknowns as above), the
source at the centre root is converted back to a zone average <R>, and the
new state is rhs + dt_m <R> (rho and rho u are the rhs: <R> is zero there).
R(U^n) at the start of a step is likewise the average of R at the centre
values of U^n.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import advection, fourth_order, network, quadrature


@dataclass
class Problem:
    dim: int
    shape: tuple            # grid extents, x first
    dx: list
    gamma: float
    net: dict
    n_nodes: int = 3
    node_type: str = "lobatto"  # or 'radau' (right Radau points, see quadrature.py)
    n_iters: int = 4
    slope: int = 1
    alpha: float = -1.0
    advection: int = 1
    newton_tol: float = 1e-13
    newton_maxiter: int = 50
    newton_extra: int = 0   # extra iterations after convergence (complex step)
    space_order: int = 2    # 4: fourth-order advective term and zone-average sources
    lnA: np.ndarray = None  # rate parameters (override the network's)
    E: np.ndarray = None

    @property
    def nspec(self):
        return self.net["nspec"]

    @property
    def ncomp(self):
        return 2 + self.dim + self.nspec

    @classmethod
    def from_workload(cls, w, **over):
        kw = dict(dim=w["dim"], shape=w["shape"], dx=w["dx"], gamma=w["gamma"],
                  net=w["network"], n_nodes=w["n_nodes"], n_iters=w["n_iters"],
                  slope=w["slope"], alpha=w["alpha"], newton_tol=w["newton_tol"],
                  newton_maxiter=w["newton_maxiter"], node_type=w.get("node_type", "lobatto"),
                  space_order=w.get("space_order", 2))
        kw.update(over)
        return cls(**kw)


@dataclass
class Stats:
    newton_total: int = 0
    solves: int = 0
    failed: int = 0
    hist: np.ndarray = field(default_factory=lambda: np.zeros(16, dtype=np.int64))

    def add(self, nu):
        ok = nu > 0
        self.solves += nu.size
        self.failed += int((~ok).sum())
        self.newton_total += int(nu[ok].sum())
        self.hist += np.bincount(np.minimum(nu[ok], 15), minlength=16)[:16]


# ------------------------------------------------------------------ pieces
def A_of(U, prob: Problem):
    if not prob.advection:
        return np.zeros_like(U)
    if prob.space_order == 4:
        return fourth_order.advective_term4(U, prob.dim, prob.dx, prob.gamma)
    return advection.advective_term(U, prob.dim, prob.dx, prob.gamma, prob.slope, prob.alpha)


def R_of_x(x, rho, prob: Problem):
    return network.source(x, rho, prob.net, prob.gamma, prob.lnA, prob.E)


def split_state(U, prob: Problem):
    """(rho [Z], momenta [d, Z], x [n, Z], KE [Z]) from U[comp, *grid]."""
    d = prob.dim
    Uf = U.reshape(U.shape[0], -1)
    rho = Uf[0]
    mom = Uf[1:1 + d]
    ke = 0.5 * (mom * mom).sum(axis=0) / rho
    x = np.concatenate([Uf[2 + d:], (Uf[1 + d] - ke)[None]], axis=0)
    return rho, mom, x, ke


def join_state(rho, mom, x, ke, prob: Problem):
    ns = prob.nspec
    Uf = np.concatenate([rho[None], mom, (x[ns] + ke)[None], x[:ns]], axis=0)
    return Uf.reshape((prob.ncomp,) + tuple(prob.shape[::-1]))


def R_full_from_x(x, prob: Problem):
    """Scatter R(x) on (rho X, rho e) into a full-length source (zeros on rho, rho u)."""
    ns = prob.nspec
    d = prob.dim
    out = np.zeros((prob.ncomp, x.shape[1]), dtype=x.dtype)
    out[1 + d] = x[ns]
    out[2 + d:] = x[:ns]
    return out.reshape((prob.ncomp,) + tuple(prob.shape[::-1]))


def R_of_state(U, prob: Problem):
    """R(U) on a full-length layout; at fourth order the zone average of R
    at the zone-centre values of U."""
    if prob.space_order == 4:
        Rc = R_of_state_point(fourth_order.to_centres(U, prob.dim), prob)
        return fourth_order.to_averages(Rc, prob.dim)
    return R_of_state_point(U, prob)


def R_of_state_point(U, prob: Problem):
    rho, _, x, _ = split_state(U, prob)
    return R_full_from_x(R_of_x(x, rho, prob), prob)


def newton_solve(b, rho, dtm, x0, prob: Problem, chunk=32768):
    """Solve x - dtm R(x; rho) = b per zone by Newton (readings in module doc).

    b, x0: [n, Z]; rho: [Z].  Returns (x [n, Z], nu [Z] int32; -1 = failed).
    """
    ns = prob.nspec
    n, Z = b.shape
    dtype = np.result_type(b, x0, rho, prob.lnA if prob.lnA is not None else 0.0,
                           prob.E if prob.E is not None else 0.0)
    x = np.array(x0, dtype=dtype, copy=True)
    nu = np.full(Z, -1, dtype=np.int32)
    eye = np.eye(n)
    for start in range(0, Z, chunk):
        sl = slice(start, min(Z, start + chunk))
        xs, bs, rs = x[:, sl], b[:, sl], rho[sl]
        scale = np.concatenate([np.broadcast_to(np.abs(rs.real), (ns, rs.size)),
                                np.abs(bs[ns].real)[None]], axis=0)
        active = np.arange(rs.size)
        conv = np.zeros(rs.size, dtype=bool)
        prev = np.zeros(rs.size)  # size of the previous step; 0 before the first

        def update(idx):
            xa = xs[:, idx]
            R, J = network.source_and_jacobian(xa, rs[idx], prob.net, prob.gamma, prob.lnA, prob.E)
            G = xa - dtm * R - bs[:, idx]
            JN = eye[None] - dtm * J
            delta = np.linalg.solve(JN, -G.T[:, :, None])[:, :, 0].T
            xs[:, idx] = xa + delta
            return np.max(np.abs(delta.real) / scale[:, idx], axis=0)

        for it in range(1, prob.newton_maxiter + 1):
            if active.size == 0:
                break
            err = update(active)
            p = prev[active]
            tol = prob.newton_tol
            # the step was small enough, or the contraction it shows bounds the
            # distance of the new iterate from the root by tol
            done = (err <= tol) | ((err < p) & (err * err <= tol * (p - err)))
            prev[active] = err
            nu[start + active[done]] = it
            conv[active[done]] = True
            active = active[~done]
        for _ in range(prob.newton_extra):
            idx = np.nonzero(conv)[0]
            if idx.size:
                update(idx)
        x[:, sl] = xs
    return x, nu


def reaction_solve(dtm, rho, b, x0, prob: Problem):
    """The implicit part of Eq. 2 alone: x - dtm R(x) = b; returns x, R(x), nu."""
    x, nu = newton_solve(b, rho, dtm, x0, prob)
    return x, R_of_x(x, rho, prob), nu


# ------------------------------------------------------------------- sweep
def node_times(prob: Problem):
    return quadrature.node_set(prob.node_type, prob.n_nodes)


def sweep(Un, A, R, U, dt, prob: Problem, stats: Stats | None = None, level=None):
    """One SDC iteration k -> k+1 over all node transitions (Eq. 2).

    Un: U^n.  A, R, U: lists over nodes of iteration-k values (A[0], R[0] are
    A(U^n), R(U^n)).  Returns the iteration-(k+1) lists (U_new, A_new, R_new).
    `level` (refined patches, see amr.py) supplies prepare(U, node), applied
    to each new node state before its advective term (ghost zones), and A(U).
    """
    tau, S = node_times(prob)
    M = prob.n_nodes - 1
    U_new, A_new, R_new = [Un], [A[0]], [R[0]]
    for m in range(M):
        dtm = (tau[m + 1] - tau[m]) * dt
        Am = A_new[m]
        integral = dt * sum(S[m, j] * (A[j] + R[j]) for j in range(M + 1))
        rhs = U_new[m] + dtm * (Am - A[m]) - dtm * R[m + 1] + integral
        _, _, x0, _ = split_state(U[m + 1], prob)
        if prob.space_order == 4:
            # the solve at zone centres, the source back to a zone average
            rho, _, b, _ = split_state(fourth_order.to_centres(rhs, prob.dim), prob)
            x, nu = newton_solve(b, rho, dtm, x0, prob)
            Ravg = fourth_order.to_averages(R_full_from_x(R_of_x(x, rho, prob), prob), prob.dim)
            U_new.append(rhs + dtm * Ravg)
            R_new.append(Ravg)
        else:
            rho, mom, b, ke = split_state(rhs, prob)
            # b holds (rhs_rhoX, rhs_rhoE - KE_new): the reacting rhs
            x, nu = newton_solve(b, rho, dtm, x0, prob)
            U_new.append(join_state(rho, mom, x, ke, prob))
            R_new.append(R_full_from_x(R_of_x(x, rho, prob), prob))
        if stats is not None:
            stats.add(nu)
        if level is not None:
            U_new[m + 1] = level.prepare(U_new[m + 1], m + 1)
            A_new.append(level.A(U_new[m + 1]))
        else:
            A_new.append(A_of(U_new[m + 1], prob))
    return U_new, A_new, R_new


def step(Un, dt, prob: Problem, A0=None, R0=None, stats: Stats | None = None):
    """One time step U^n -> U^{n+1} = U^{M,(K)}; returns (U^{n+1}, A^M, R^M)."""
    M = prob.n_nodes - 1
    A0 = A_of(Un, prob) if A0 is None else A0
    R0 = R_of_state(Un, prob) if R0 is None else R0
    U = [Un] * (M + 1)
    A = [A0] * (M + 1)
    R = [R0] * (M + 1)
    for _ in range(prob.n_iters):
        U, A, R = sweep(Un, A, R, U, dt, prob, stats)
    return U[M], A[M], R[M]


def run(U0, dt, nsteps, prob: Problem, stats: Stats | None = None):
    """nsteps steps; the last node's sources become the next step's node 0."""
    U, A0, R0 = U0, None, None
    for _ in range(nsteps):
        U, A0, R0 = step(U, dt, prob, A0, R0, stats)
    return U


def energy_released(U0, UN, prob: Problem):
    """J_E = dV sum_z sum_i q_i [rhoX_i(t0) - rhoX_i(tN)] (total reaction energy)."""
    d = prob.dim
    dV = float(np.prod(prob.dx))
    q = prob.net["q"]
    s0 = U0.reshape(U0.shape[0], -1)[2 + d:]
    sN = UN.reshape(UN.shape[0], -1)[2 + d:]
    return dV * np.sum(q[:, None] * (s0 - sN))
