"""GPU parity: every C-ABI entry point against the CPU oracle on the same
seeded inputs (paper Sec. 2, Eq. 1 and Eq. 2).

Grids span several 256-zone blocks and end in a ragged tail.  The bar is the
normwise relative error per component: <= 1e-10 in FP64, <= 1e-8 for the
mixed mode (FP32 Newton matrix and LU, FP64 residual and update).
"""
import dataclasses

import numpy as np
import pytest

import sdc_inputs as si
from oracle import sdc as osdc
from tests.helpers import TOL_FP64, TOL_MIXED, rel_err_per_component, to_gpu, to_np

pytestmark = pytest.mark.gpu

SHAPES = {"chain1d": (64,), "net2d": (40, 28), "net3d": (12, 10, 9), "adjoint2d": (24, 20)}


def make(name, shape=None, **over):
    from paper_1910_12578_amd import SDC, config_from_workload
    w = si.workload(name, shape=shape or SHAPES[name])
    prob_over = {k: v for k, v in over.items() if k in ("n_nodes", "n_iters", "slope", "alpha", "advection",
                                                         "newton_maxiter", "newton_tol", "node_type")}
    prob = osdc.Problem.from_workload(w, **prob_over)
    cfg = config_from_workload(w, **over)
    return w, prob, SDC(cfg, w["network"])


def reacting(Rfull, dim):
    """Oracle full-length source -> reacting layout (species, energy)."""
    Rf = Rfull.reshape(Rfull.shape[0], -1)
    return np.concatenate([Rf[2 + dim:], Rf[1 + dim:2 + dim]], axis=0)


def assert_close(a, ref, tol, what):
    e = rel_err_per_component(a, ref)
    print(f"{what}: max rel err per component {e.max():.3e}")
    assert np.all(e <= tol), (what, e)


@pytest.mark.parametrize("name", ["chain1d", "net2d", "net3d"])
@pytest.mark.parametrize("slope,alpha", [(1, -1.0), (0, -1.0), (0, 1.9)])
def test_advective_term(name, slope, alpha):
    w, prob, h = make(name, slope=slope, alpha=alpha)
    U = w["U0"]
    A = to_np(h.advective_term(to_gpu(U.reshape(U.shape[0], -1))))
    ref = osdc.A_of(U, prob).reshape(U.shape[0], -1)
    assert_close(A, ref, 1e-11, f"A {name} slope={slope} alpha={alpha}")


@pytest.mark.parametrize("shape", [(256, 2, 3), (257, 3, 2), (384, 2, 3), (512, 3, 2), (513, 2, 2),
                                   (5, 7, 33), (64, 5, 4)])
@pytest.mark.parametrize("slope", [1, 0])
def test_advective_term_3d_edge_shapes(shape, slope):
    """3D grids at the edges of the row kernel: a full 256-zone row per block
    with periodic images in y and z (n = 2, 3), rows of 257..512 zones (the
    512-thread blocks, with idle lanes and full), a row longer than any block
    (the zone-per-thread kernel), many rows per block with a z extent above
    one chunk, and several rows per block."""
    w, prob, h = make("net3d", shape=shape, slope=slope)
    U = w["U0"]
    A = to_np(h.advective_term(to_gpu(U.reshape(U.shape[0], -1))))
    ref = osdc.A_of(U, prob).reshape(U.shape[0], -1)
    assert_close(A, ref, 1e-11, f"A {shape} slope={slope}")


@pytest.mark.parametrize("name", ["chain1d", "net2d", "net3d"])
def test_source(name):
    w, prob, h = make(name)
    U = w["U0"]
    R = to_np(h.source(to_gpu(U.reshape(U.shape[0], -1))))
    ref = reacting(osdc.R_of_state(U, prob), prob.dim)
    assert_close(R, ref, 1e-11, f"R {name}")


@pytest.mark.parametrize("name", ["chain1d", "net2d", "net3d"])
@pytest.mark.parametrize("precision", [0, 1])
def test_reaction_solve(name, precision):
    w, prob, h = make(name, precision=precision)
    rho, _, x0, _ = osdc.split_state(w["U0"], prob)
    g = si.rng(7)
    b = x0 * (1.0 + 0.05 * g.uniform(-1, 1, x0.shape))
    dtm = 2.0 * w["dt"]
    x, R, nu = osdc.reaction_solve(dtm, rho, b, x0, prob)
    xg, Rg, nug = h.reaction_solve(dtm, to_gpu(rho), to_gpu(b), to_gpu(x0))
    tol = TOL_FP64 if precision == 0 else TOL_MIXED
    assert_close(to_np(xg), x, tol, f"x {name} p{precision}")
    # R at the root: the roots agree to the Newton tolerance, and R amplifies
    # that difference by |dR/dx| |x| / |R|, large for the stiff rates; so R is
    # checked as a function at the GPU's own root (FP64 in both modes), at
    # the FP64 bar
    R_at_root = osdc.R_of_x(to_np(xg), rho, prob)
    assert_close(to_np(Rg), R_at_root, TOL_FP64, f"R(x) {name} p{precision}")
    nug = to_np(nug)
    assert np.all(nug > 0) and np.all(nu > 0)
    if precision == 0:
        assert np.mean(nug == nu) > 0.97 and np.max(np.abs(nug - nu)) <= 1
    else:
        # FP32 factors: Newton becomes iterative refinement, a few more steps
        print(f"mixed: mean Newton {nug.mean():.2f} vs FP64 oracle {nu.mean():.2f}")
        assert np.max(np.abs(nug - nu)) <= 3
    st = h.stats()
    assert st["solves"] == nu.size and st["failed"] == 0 and st["nonfinite"] == 0
    assert st["iters"] == int(nug.sum()) and sum(st["hist"]) == nu.size


def test_sweep_iterations_match():
    w, prob, h = make("net2d")
    U0 = w["U0"]
    nc = U0.shape[0]
    dt = w["dt"]
    nodes = h.alloc_nodes()
    nodes["U"][0].copy_(to_gpu(U0.reshape(nc, -1)))
    h.advective_term(nodes["U"][0], nodes["A"][0])
    h.source(nodes["U"][0], nodes["R"][0])
    A0 = osdc.A_of(U0, prob)
    R0 = osdc.R_of_state(U0, prob)
    U, A, R = [U0] * 3, [A0] * 3, [R0] * 3
    for k in range(3):
        h.sweep(dt, k, nodes)
        U, A, R = osdc.sweep(U0, A, R, U, dt, prob)
        for m in (1, 2):
            assert_close(to_np(nodes["U"][m]), U[m].reshape(nc, -1), TOL_FP64, f"U^{m} k={k + 1}")
            assert_close(to_np(nodes["A"][m]), A[m].reshape(nc, -1), TOL_FP64, f"A^{m} k={k + 1}")
            assert_close(to_np(nodes["R"][m]), reacting(R[m], 2), TOL_FP64, f"R^{m} k={k + 1}")


@pytest.mark.parametrize("name,nsteps,over", [
    ("chain1d", 10, {}),
    ("net2d", 2, {}),
    ("net3d", 1, {}),
    ("adjoint2d", 3, {}),
    ("net2d", 1, {"n_nodes": 2, "n_iters": 2}),
    ("net2d", 1, {"n_nodes": 4, "n_iters": 3}),
    ("net2d", 1, {"n_nodes": 5, "n_iters": 2}),
    ("net2d", 1, {"advection": 0}),
    # right Radau node sets (1..4 Radau points after tau_0 = 0)
    ("net2d", 1, {"node_type": "radau", "n_nodes": 2, "n_iters": 2}),
    ("net2d", 2, {"node_type": "radau", "n_nodes": 3, "n_iters": 4}),
    ("net2d", 1, {"node_type": "radau", "n_nodes": 4, "n_iters": 3}),
    ("net2d", 1, {"node_type": "radau", "n_nodes": 5, "n_iters": 2}),
    ("net3d", 1, {"node_type": "radau", "n_nodes": 3, "n_iters": 4}),
    ("chain1d", 10, {"node_type": "radau"}),
])
def test_step_matches_oracle(name, nsteps, over):
    w, prob, h = make(name, **over)
    U0 = w["U0"]
    nc = U0.shape[0]
    Ug = to_gpu(U0.reshape(nc, -1))
    h.step(w["dt"], nsteps, Ug)
    st = osdc.Stats()
    ref = osdc.run(U0, w["dt"], nsteps, prob, st).reshape(nc, -1)
    assert_close(to_np(Ug), ref, TOL_FP64, f"step {name} x{nsteps} {over}")
    s = h.stats()
    assert s["solves"] == st.solves and s["failed"] == 0 and s["nonfinite"] == 0
    # Newton iteration counts agree up to rare one-off stops at the tolerance
    assert abs(s["iters"] - st.newton_total) <= max(2, st.newton_total // 500)


@pytest.mark.parametrize("name,nsteps", [("net2d", 2), ("net3d", 1)])
def test_mixed_precision_step(name, nsteps):
    w, prob, h = make(name, precision=1)
    U0 = w["U0"]
    nc = U0.shape[0]
    Ug = to_gpu(U0.reshape(nc, -1))
    h.step(w["dt"], nsteps, Ug)
    ref = osdc.run(U0, w["dt"], nsteps, prob).reshape(nc, -1)
    e = rel_err_per_component(to_np(Ug), ref)
    print("mixed per-component error vs FP64 oracle:", " ".join(f"{v:.2e}" for v in e))
    assert np.all(e <= TOL_MIXED)
    assert h.stats()["failed"] == 0


def test_pivoting_fallback_path():
    """pivot_threshold > 1 sends every solve to the dense partially pivoted path."""
    w, prob, h = make("net2d", pivot_threshold=2.0)
    U0 = w["U0"]
    nc = U0.shape[0]
    Ug = to_gpu(U0.reshape(nc, -1))
    h.step(w["dt"], 1, Ug)
    ref = osdc.run(U0, w["dt"], 1, prob).reshape(nc, -1)
    assert_close(to_np(Ug), ref, TOL_FP64, "dense pivoted path")
    s = h.stats()
    assert s["fallbacks"] == s["solves"] and s["failed"] == 0


def test_unconverged_zones_are_flagged():
    w, prob, h = make("net2d", newton_maxiter=1)
    rho, _, x0, _ = osdc.split_state(w["U0"], prob)
    xg, Rg, nug = h.reaction_solve(3 * w["dt"], to_gpu(rho), to_gpu(x0 * 1.01), to_gpu(x0))
    p1 = dataclasses.replace(prob, newton_maxiter=1)
    x, _, nu = osdc.reaction_solve(3 * w["dt"], rho, x0 * 1.01, x0, p1)
    assert np.all(to_np(nug) == -1) and np.all(nu == -1)
    assert_close(to_np(xg), x, TOL_FP64, "kept last iterate")
    s = h.stats()
    assert s["failed"] == s["solves"] == x.shape[1]
    assert h.check()[0] == 4  # SDC_ERR_NEWTON
    h.stats_reset()
    assert h.check() == (0, "")


def test_non_finite_zone_is_counted_not_fatal():
    w, prob, h = make("net2d")
    rho, _, x0, _ = osdc.split_state(w["U0"], prob)
    b = x0.copy()
    b[-1, 5] = -1.0  # negative internal energy: T < 0, log(T) is NaN
    xg, Rg, nug = h.reaction_solve(w["dt"], to_gpu(rho), to_gpu(b), to_gpu(x0))
    nug = to_np(nug)
    assert nug[5] == -1 and np.all(np.delete(nug, 5) > 0)
    s = h.stats()
    assert s["nonfinite"] >= 1 and s["failed"] == 1
    assert h.check()[0] == 5  # SDC_ERR_NONFINITE
    ok = np.ones(b.shape[1], bool)
    ok[5] = False
    x, _, _ = osdc.reaction_solve(w["dt"], rho[ok], b[:, ok], x0[:, ok], prob)
    assert_close(to_np(xg)[:, ok], x, TOL_FP64, "finite zones")


def test_run_twice_is_bitwise_identical():
    w, prob, h = make("net3d")
    nc = w["U0"].shape[0]
    a = to_gpu(w["U0"].reshape(nc, -1))
    b = a.clone()
    work = h.alloc_nodes()
    h.step(w["dt"], 1, a, work)
    h.step(w["dt"], 1, b, work)
    assert bool((a == b).all())


def test_bad_arguments_raise():
    import torch
    from paper_1910_12578_amd import SDCError
    w, prob, h = make("chain1d")
    U = to_gpu(w["U0"])
    with pytest.raises(SDCError):
        h.step(-1.0, 1, U)
    with pytest.raises(ValueError):
        h.advective_term(U[:, :10].contiguous())
    with pytest.raises(TypeError):
        h.advective_term(U.float())


@pytest.mark.parametrize("name", ["chain1d", "net2d"])
def test_graph_replay_matches_eager_bitwise(name):
    """Captured steps replayed several times, with eager work in between,
    equal plain launches bit for bit after every call."""
    import torch
    w, prob, hg = make(name, graph=1)
    _, _, he = make(name, graph=0)
    nc = w["U0"].shape[0]
    a = to_gpu(w["U0"].reshape(nc, -1))
    b = a.clone()
    wa, wb = hg.alloc_nodes(), he.alloc_nodes()
    for rep in range(4):
        hg.step(w["dt"], 2 + rep % 2, a, wa)
        scratch = torch.randn(1000, device="cuda").abs().sum()  # unrelated eager work
        he.step(w["dt"], 2 + rep % 2, b, wb)
        torch.cuda.synchronize()
        assert bool((a == b).all()), f"replay {rep} differs"
        assert bool(torch.isfinite(scratch))
    sa, sb = hg.stats(), he.stats()
    assert sa == sb


def test_graph_step_latency_report():
    """Per-step wall time of the 64-zone chain with and without graphs (report)."""
    import time
    import torch
    w, prob, hg = make("chain1d", graph=1)
    _, _, he = make("chain1d", graph=0)
    nc = w["U0"].shape[0]
    for h, label in ((he, "launches"), (hg, "graph")):
        U = to_gpu(w["U0"].reshape(nc, -1))
        work = h.alloc_nodes()
        h.step(w["dt"], 10, U, work)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.step(w["dt"], 200, U, work)
        torch.cuda.synchronize()
        print(f"chain1d {label}: {1e6 * (time.perf_counter() - t0) / 200:.1f} us per step")
