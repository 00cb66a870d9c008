"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module draws reaction networks and initial states from fixed seeds and
converts the drawn primitive fields (density, velocity, pressure, mass
fractions) to the conserved vector U = (rho, rho*u_1..rho*u_d, rho*E,
rho*X_1..rho*X_Ns).  It contains none of the SDC method's arithmetic (no
advective term, no reaction source, no quadrature, no Newton solve), so both
the oracle and the GPU path can consume it without sharing method code.

The paper (Sec. 2, Eq. 1) works with a vector of conserved quantities and a
stiff nuclear network; it gives no data, so the workloads below are synthetic
stand-ins whose sizes follow the five benchmark configurations:

  chain1d   1D, 64 zones, 4-species linear chain A->B->C->D, 2 nodes, K=2
  net2d     2D 512^2, 7 species / 10 reactions, 3 nodes, K=4
  net3d     3D 256^3, 13 species / 20 reactions, 3 nodes, K=4
  boxes     4096 periodic 3D boxes with edges in {8,16,32,64}, 13/20 network
  adjoint2d 2D 256^2, 7/10 network, smooth mode, 20 steps

Units: gamma-law gas with p = rho*T (so c_v = 1/(gamma-1)), T0 = 1, p0 = 1.
"""
from __future__ import annotations

import math
import numpy as np

GAMMA = 1.4

# fixed seeds of every workload
SEEDS = {
    "chain1d_state": 101,
    "net7_network": 202,
    "net2d_state": 203,
    "net13_network": 302,
    "net3d_state": 303,
    "boxes_state": 403,
    "adjoint2d_state": 503,
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------- networks
def chain_network(rates=(1.0, 1.0e3, 1.0e6), q=(0.3, 0.2, 0.1, 0.0)) -> dict:
    """Linear chain A->B->C->D with constant first-order rates.

    Constant rates are expressed in the Arrhenius form k = exp(lnA + b lnT - E/T)
    with b = E = 0 and lnA = ln k.
    """
    nspec = len(q)
    nreact = nspec - 1
    reactants = np.full((nreact, 2), -1, dtype=np.int32)
    stoich = np.zeros((nreact, nspec))
    for r in range(nreact):
        reactants[r, 0] = r
        stoich[r, r] = -1.0
        stoich[r, r + 1] = 1.0
    return {
        "nspec": nspec,
        "nreact": nreact,
        "reactants": reactants,
        "stoich": stoich,
        "lnA": np.log(np.asarray(rates, dtype=float)),
        "b": np.zeros(nreact),
        "E": np.zeros(nreact),
        "q": np.asarray(q, dtype=float),
    }


def random_network(nspec: int, nreact: int, seed: int, q_max: float = 0.25,
                   log10A=(2.0, 8.0), E=(5.0, 40.0), b=(0.0, 2.0),
                   T0: float = 1.0) -> dict:
    """Synthetic Arrhenius network drawn from `seed` (no physical rate data).

    Each reaction is, with probability 1/2, unimolecular i -> j (i < j,
    stoichiometry -1/+1, rate rho*w = k x_i) or bimolecular i + j -> k
    (i < j < k, stoichiometry -1/-1/+2, rate rho*w = k x_i x_j), with
    x_i = rho X_i.  k = A T^b exp(-E/T), log10 A ~ U[2,8], E ~ U[5,40] T0,
    b ~ U[0,2].  Binding energies q_i ~ U[0, q_max] sorted in descending
    order, so every reaction releases energy.
    """
    g = rng(seed)
    reactants = np.full((nreact, 2), -1, dtype=np.int32)
    stoich = np.zeros((nreact, nspec))
    for r in range(nreact):
        if nspec < 3 or g.random() < 0.5:
            i, j = np.sort(g.choice(nspec, size=2, replace=False))
            reactants[r, 0] = i
            stoich[r, i] = -1.0
            stoich[r, j] = 1.0
        else:
            i, j, k = np.sort(g.choice(nspec, size=3, replace=False))
            reactants[r] = (i, j)
            stoich[r, i] = -1.0
            stoich[r, j] = -1.0
            stoich[r, k] = 2.0
    log10A_r = g.uniform(*log10A, size=nreact)
    E_r = g.uniform(*E, size=nreact) * T0
    b_r = g.uniform(*b, size=nreact)
    q = np.sort(g.uniform(0.0, q_max, size=nspec))[::-1].copy()
    return {
        "nspec": nspec,
        "nreact": nreact,
        "reactants": reactants,
        "stoich": stoich,
        "lnA": log10A_r * math.log(10.0),
        "b": b_r,
        "E": E_r,
        "q": q,
    }


# ------------------------------------------------------------------ states
def conserved_from_primitive(rho, u, p, X, gamma=GAMMA) -> np.ndarray:
    """Stack (rho, rho u_d, rho E, rho X_s) into U[comp, *grid] (x fastest)."""
    dim = len(u)
    nspec = X.shape[0]
    U = np.empty((2 + dim + nspec,) + rho.shape, dtype=np.result_type(rho, p, X, *u))
    U[0] = rho
    ke = np.zeros_like(rho)
    for d in range(dim):
        U[1 + d] = rho * u[d]
        ke += 0.5 * rho * u[d] * u[d]
    U[1 + dim] = p / (gamma - 1.0) + ke
    U[2 + dim:] = rho[None] * X
    return U


def cfl_dt(rho, u, p, dx, gamma=GAMMA, cfl=0.5) -> float:
    """dt = cfl / max_z sum_d (|u_d| + c)/dx_d on the drawn primitive state."""
    c = np.sqrt(gamma * p / rho)
    s = np.zeros_like(rho)
    for d in range(len(u)):
        s += (np.abs(u[d]) + c) / dx[d]
    return float(cfl / s.max())


def max_signal_speed(rho, u, p, gamma=GAMMA) -> float:
    c = np.sqrt(gamma * p / rho)
    return float(max((np.abs(u[d]) + c).max() for d in range(len(u))))


def _centers(n):
    return (np.arange(n) + 0.5) / n


def _mesh(shape_xfirst):
    """Zone-centre coordinates of the unit box; returns [x, y, z] arrays shaped
    like the grid in C order (slowest ... fastest = z ... x)."""
    axes = [_centers(n) for n in shape_xfirst]
    grids = np.meshgrid(*axes[::-1], indexing="ij")  # slowest first
    return grids[::-1]


def chain1d_state(n=64, seed=SEEDS["chain1d_state"], gamma=GAMMA):
    """1D smooth density/velocity, uniform pressure, pure species A."""
    g = rng(seed)
    a_rho = g.uniform(0.1, 0.3)
    a_u = g.uniform(0.05, 0.2)
    ph_rho, ph_u = g.uniform(0.0, 1.0, size=2)
    (x,) = _mesh((n,))
    rho = 1.0 + a_rho * np.sin(2 * np.pi * (x + ph_rho))
    u = [a_u * np.sin(2 * np.pi * (x + ph_u))]
    p = np.ones_like(rho)
    X = np.zeros((4,) + rho.shape)
    X[0] = 1.0
    return rho, u, p, X


def reactive_state(shape_xfirst, nspec, seed, perturb=0.0, vel=0.1,
                   lognormal_sigma=None, gamma=GAMMA):
    """Smooth temperature background, isobaric density, smooth velocity.

    T = 1 + 0.1 prod_d sin 2pi(x_d + phi_d), optionally times (1 + perturb*xi)
    with xi ~ U[-1,1] per zone, or T = exp(sigma*zeta) with zeta ~ N(0,1).
    rho = p/T with p = 1.  u_d = vel sin 2pi(x_{d+1} + psi_d).
    X_1 = 0.9 and the remaining 0.1 split by per-zone U[0,1] weights.
    """
    g = rng(seed)
    dim = len(shape_xfirst)
    xs = _mesh(shape_xfirst)
    phi = g.uniform(0.0, 1.0, size=dim)
    psi = g.uniform(0.0, 1.0, size=dim)
    gshape = xs[0].shape
    if lognormal_sigma is not None:
        T = np.exp(lognormal_sigma * g.standard_normal(gshape))
    else:
        prod = np.ones(gshape)
        for d in range(dim):
            prod = prod * np.sin(2 * np.pi * (xs[d] + phi[d]))
        T = 1.0 + 0.1 * prod
        if perturb:
            T = T * (1.0 + perturb * g.uniform(-1.0, 1.0, size=gshape))
    p = np.ones(gshape)
    rho = p / T
    u = [vel * np.sin(2 * np.pi * (xs[(d + 1) % dim] + psi[d])) for d in range(dim)]
    w = g.uniform(0.0, 1.0, size=(nspec - 1,) + gshape)
    X = np.empty((nspec,) + gshape)
    X[0] = 0.9
    X[1:] = 0.1 * w / w.sum(axis=0, keepdims=True)
    return rho, u, p, X


def box_extents(nbox=4096, seed=SEEDS["boxes_state"], choices=(8, 16, 32, 64)):
    """[nbox, 3] box edges (x, y, z), each edge iid uniform over `choices`."""
    g = rng(seed)
    return g.choice(np.asarray(choices, dtype=np.int64), size=(nbox, 3))


def box_state(extents, nspec, seed=SEEDS["boxes_state"] + 1, sigma=0.3, vel=0.05,
              gamma=GAMMA):
    """Concatenated SoA state of independent periodic boxes.

    Per zone T = exp(sigma zeta), zeta ~ N(0,1) (the lognormal of the batched
    workload, untruncated: the draw of the standard seed spans |zeta| <= 5.95,
    T from 0.17 to 5.96); isobaric rho = 1/T; velocity
    0.05 sin of box-local coordinates; X as in `reactive_state`.  Returns
    (U [n_c, Ztot], offsets [nbox+1]).
    """
    g = rng(seed)
    dim = 3
    nzones = np.prod(extents, axis=1)
    offsets = np.concatenate([[0], np.cumsum(nzones)]).astype(np.int64)
    ztot = int(offsets[-1])
    # lognormal temperature
    zeta = g.standard_normal(ztot)
    T = np.exp(sigma * zeta)
    rho = 1.0 / T
    p = np.ones(ztot)
    u = [np.empty(ztot) for _ in range(dim)]
    for bi, ext in enumerate(extents):
        xs = [c.ravel() for c in _mesh(tuple(int(e) for e in ext))]
        sl = slice(offsets[bi], offsets[bi + 1])
        for d in range(dim):
            u[d][sl] = vel * np.sin(2 * np.pi * xs[(d + 1) % dim])
    w = g.uniform(0.0, 1.0, size=(nspec - 1, ztot))
    X = np.empty((nspec, ztot))
    X[0] = 0.9
    X[1:] = 0.1 * w / w.sum(axis=0, keepdims=True)
    U = conserved_from_primitive(rho, u, p, X, gamma)
    return U, offsets, (rho, u, p)


# ---------------------------------------------------------------- workloads
FULL_SHAPES = {"chain1d": (64,), "net2d": (512, 512), "adjoint2d": (256, 256), "net3d": (256, 256, 256)}


def workload(name: str, shape=None, steps=None) -> dict:
    """Everything one run needs: grid, network, U0 [n_c, *grid], dt and knobs.

    `shape` overrides the grid (x first) for reduced-size parity cases that
    keep the workload's recipe.  The time step is always the CFL step of the
    full-size grid (the drawn state's signal speeds with the full grid's dx),
    so reduced cases see the same reaction stiffness per step as the real run.
    """
    if name == "chain1d":
        shape = shape or (64,)
        net = chain_network()
        rho, u, p, X = chain1d_state(shape[0])
        d = dict(n_nodes=2, n_iters=2, steps=10, slope=1, cfl=0.5)
    elif name in ("net2d", "adjoint2d"):
        shape = shape or ((512, 512) if name == "net2d" else (256, 256))
        net = random_network(7, 10, SEEDS["net7_network"])
        seed = SEEDS["net2d_state"] if name == "net2d" else SEEDS["adjoint2d_state"]
        rho, u, p, X = reactive_state(shape, 7, seed)
        if name == "net2d":
            d = dict(n_nodes=3, n_iters=4, steps=10, slope=1, cfl=0.5)
        else:
            d = dict(n_nodes=3, n_iters=4, steps=20, slope=0, cfl=0.4)
    elif name == "net3d":
        shape = shape or (256, 256, 256)
        net = random_network(13, 20, SEEDS["net13_network"])
        rho, u, p, X = reactive_state(shape, 13, SEEDS["net3d_state"], perturb=0.2)
        d = dict(n_nodes=3, n_iters=4, steps=10, slope=1, cfl=0.5)
    else:
        raise ValueError(f"unknown workload {name!r}")
    dim = len(shape)
    dx = [1.0 / n for n in shape]
    dx_full = [1.0 / n for n in FULL_SHAPES[name]]
    U0 = conserved_from_primitive(rho, u, p, X)
    alpha = -1.0
    if d["slope"] == 0:
        alpha = 1.2 * max_signal_speed(rho, u, p)
    out = dict(name=name, dim=dim, shape=tuple(shape), dx=dx, gamma=GAMMA,
               network=net, U0=U0, dt=cfl_dt(rho, u, p, dx_full, cfl=d["cfl"]),
               alpha=alpha, newton_tol=1e-13, newton_maxiter=50, **d)
    if steps is not None:
        out["steps"] = steps
    return out


def boxes_workload(nbox=4096, choices=(8, 16, 32, 64), sigma=0.3, seed=SEEDS["boxes_state"],
                   dt_factor=0.4, q_max=0.85) -> dict:
    """Batched AMR-like boxes: `nbox` independent periodic 3D boxes with edges
    iid uniform over `choices`, the 13-species network, per-zone lognormal
    temperature (so Newton iteration counts spread), dx = 1/256 in every box.

    The network is the 13-species one of the other 3D workloads with binding
    energies drawn up to `q_max` = 0.85 (3.4 times theirs; the rates are the
    same draws): the heat a hot zone releases within a step raises its
    temperature and its rates, so in the first step its Newton solves take up
    to 8 iterations while most take 2 or 3.  Hotter settings (q_max 1.0 at
    this step) spread the counts to 11 but let the hottest zones of the full
    draw run away within a step, where Newton stops converging.  The step is
    `dt_factor` times the CFL step (a burning-limited step) and the nodes are
    tau_0 = 0 plus two right Radau points (K = 4): in the hot tail of the
    lognormal (T up to 6) the Gauss-Lobatto sweeps, whose fixed point does not
    damp stiff modes, drive mass fractions negative and some Newton solves stop
    converging, and the advective term then carries the failure to neighbouring
    zones; the Radau sweeps converge in every zone.

    U0 is the concatenated SoA state [n_c, sum of box zones]; box_off holds the
    zone offsets of the boxes.
    """
    net = random_network(13, 20, SEEDS["net13_network"], q_max=q_max)
    ext = box_extents(nbox, seed, choices)
    U0, offsets, (rho, u, p) = box_state(ext, 13, seed + 1, sigma=sigma)
    dx = [1.0 / 256] * 3
    return dict(name="boxes", dim=3, shape=None, box_n=ext, box_off=offsets, dx=dx, gamma=GAMMA,
                network=net, U0=U0, dt=dt_factor * cfl_dt(rho, u, p, dx, cfl=0.5), alpha=-1.0, n_nodes=3,
                node_type="radau", n_iters=4, steps=10, slope=1, cfl=0.5, newton_tol=1e-13, newton_maxiter=50)
