"""GPU parity of the fourth-order method in space (paper Sec. 2: Simpson's
rule with McCorquodale and Colella's reconstruction) against the oracle.

Covers the fourth-order advective term, the zone-average reactive source,
whole steps (the zone-centre Newton solve and the average store inside every
transition) in 1D, 2D and 3D, mixed precision, right Radau nodes, and the
configurations the mode rejects.  Grids span several 256-zone blocks and end
in ragged tails; the bar is the FP64 one (1e-10 normwise per component;
1e-11 for A alone) and 1e-8 in mixed precision.
"""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import sdc as osdc
from tests.helpers import TOL_FP64, TOL_MIXED, rel_err_per_component, to_gpu, to_np

pytestmark = pytest.mark.gpu

SHAPES = {"chain1d": (64,), "net2d": (40, 28), "net3d": (12, 10, 9)}
PROB_KEYS = ("n_nodes", "n_iters", "advection", "node_type", "space_order")


def make(name, shape=None, **over):
    from paper_1910_12578_amd import SDC, config_from_workload
    over.setdefault("space_order", 4)
    w = si.workload(name, shape=shape or SHAPES[name])
    prob = osdc.Problem.from_workload(w, **{k: v for k, v in over.items() if k in PROB_KEYS})
    return w, prob, SDC(config_from_workload(w, **over), w["network"])


def assert_close(a, ref, tol, what):
    e = rel_err_per_component(a, ref)
    print(f"{what}: max rel err per component {e.max():.3e}", flush=True)
    assert np.all(e <= tol), (what, e)


def reacting(Rfull, dim):
    Rf = Rfull.reshape(Rfull.shape[0], -1)
    return np.concatenate([Rf[2 + dim:], Rf[1 + dim:2 + dim]], axis=0)


@pytest.mark.parametrize("name,shape", [("chain1d", None), ("net2d", None), ("net3d", None),
                                        ("net2d", (5, 3)), ("net3d", (4, 2, 3))])
def test_advective_term4(name, shape):
    w, prob, h = make(name, shape)
    U = w["U0"]
    A = to_np(h.advective_term(to_gpu(U.reshape(U.shape[0], -1))))
    ref = osdc.A_of(U, prob).reshape(U.shape[0], -1)
    assert_close(A, ref, 1e-11, f"A4 {name} {shape}")
    h.close()


@pytest.mark.parametrize("name", ["chain1d", "net2d", "net3d"])
def test_average_source(name):
    w, prob, h = make(name)
    U = w["U0"]
    R = to_np(h.source(to_gpu(U.reshape(U.shape[0], -1))))
    ref = reacting(osdc.R_of_state(U, prob), prob.dim)
    assert_close(R, ref, 1e-11, f"<R> {name}")
    h.close()


@pytest.mark.parametrize("name,nsteps,over", [
    ("chain1d", 10, {}),
    ("net2d", 2, {}),
    ("net3d", 1, {}),
    ("net2d", 1, {"n_nodes": 2, "n_iters": 2}),
    ("net2d", 1, {"advection": 0}),
    ("net2d", 1, {"node_type": "radau", "n_nodes": 3, "n_iters": 4}),
])
def test_step4_matches_oracle(name, nsteps, over):
    w, prob, h = make(name, **over)
    U0 = w["U0"]
    nc = U0.shape[0]
    Ug = to_gpu(U0.reshape(nc, -1))
    print(f"[order4] {name} x{nsteps} {over}", flush=True)
    h.step(w["dt"], nsteps, Ug)
    st = osdc.Stats()
    ref = osdc.run(U0, w["dt"], nsteps, prob, st).reshape(nc, -1)
    assert_close(to_np(Ug), ref, TOL_FP64, f"step4 {name} x{nsteps} {over}")
    s = h.stats()
    assert s["solves"] == st.solves and s["failed"] == 0 and s["nonfinite"] == 0
    assert abs(s["iters"] - st.newton_total) <= max(2, st.newton_total // 500)
    h.close()


def test_step4_mixed_precision():
    w, prob, h = make("net2d", precision=1)
    U0 = w["U0"]
    nc = U0.shape[0]
    Ug = to_gpu(U0.reshape(nc, -1))
    h.step(w["dt"], 2, Ug)
    ref = osdc.run(U0, w["dt"], 2, prob).reshape(nc, -1)
    assert_close(to_np(Ug), ref, TOL_MIXED, "step4 mixed")
    h.close()


def test_step4_graph_replay_matches_launches():
    """Captured steps replay the fourth-order kernels bit for bit."""
    w, prob, h = make("net2d")
    wg, _, hg = make("net2d", graph=1)
    nc = w["U0"].shape[0]
    U = to_gpu(w["U0"].reshape(nc, -1))
    Ug = U.clone()
    for _ in range(3):
        h.step(w["dt"], 1, U)
        hg.step(w["dt"], 1, Ug)
        assert np.array_equal(to_np(U), to_np(Ug))
    h.close()
    hg.close()


def test_fourth_order_rejects_boxes_and_adjoint():
    from paper_1910_12578_amd import SDC, SDCError, config_from_workload
    wb = si.boxes_workload(nbox=3, choices=(8,))
    with pytest.raises(SDCError, match="SDC_ERR_UNSUPPORTED"):
        SDC(config_from_workload(wb, space_order=4), wb["network"])
    w, _, h = make("net2d", slope=0, alpha=2.0)
    nc = w["U0"].shape[0]
    U = to_gpu(w["U0"].reshape(nc, -1))
    with pytest.raises(SDCError, match="SDC_ERR_UNSUPPORTED"):
        h.step_adjoint(w["dt"], U, U.clone())
    h.close()


def test_step4_schedules_bitwise_identical():
    """The Newton schedules (register budget, iteration cap with the deferred
    finish kernel) only move where a zone's iterations run, also in the
    fourth-order transitions' centre solve: every one gives the default bits."""
    import torch
    w, prob, h = make("net2d")
    nc = w["U0"].shape[0]

    def one():
        U = to_gpu(w["U0"].reshape(nc, -1))
        h.stats_reset()
        h.step(w["dt"], 2, U)
        return U, h.stats()

    ref, sref = one()
    for sched in [(1, 0, 0, 0), (0, 1, 0, 0), (1, 2, 0, 0), (0, 3, 0, 0)]:
        h.set_schedule(*sched)
        U, s = one()
        assert bool(torch.equal(U, ref)), sched
        assert s == sref, sched
    h.close()
