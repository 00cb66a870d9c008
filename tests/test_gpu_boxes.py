"""Batched AMR-like boxes: one launch per kernel over many independent periodic
boxes of uneven size must equal the oracle run box by box (single-level
boxes, paper Sec. 2; every box is its own periodic grid)."""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import sdc as osdc
from tests.helpers import TOL_FP64, TOL_MIXED, rel_err_per_component, to_gpu, to_np

pytestmark = pytest.mark.gpu


def small_boxes(nbox=9, choices=(2, 4, 6), seed=77):
    w = si.boxes_workload(nbox=nbox, choices=choices, seed=seed)
    return w


def oracle_boxes(w, fn):
    """Apply fn(U_box, problem) to every box and concatenate."""
    out = []
    for b, ext in enumerate(w["box_n"]):
        lo, hi = w["box_off"][b], w["box_off"][b + 1]
        shape = tuple(int(e) for e in ext)
        Ub = np.ascontiguousarray(w["U0"][:, lo:hi]).reshape((w["U0"].shape[0],) + shape[::-1])
        prob = osdc.Problem.from_workload(dict(w, shape=shape))
        out.append(fn(Ub, prob).reshape(w["U0"].shape[0], -1))
    return np.concatenate(out, axis=1)


def make(w, **over):
    from paper_1910_12578_amd import SDC, config_from_workload
    return SDC(config_from_workload(w, **over), w["network"])


def test_box_table_layout():
    w = small_boxes()
    sizes = np.prod(w["box_n"], axis=1)
    assert w["U0"].shape[1] == sizes.sum() and np.all(np.diff(w["box_off"]) == sizes)
    assert w["U0"].shape[1] % 256 != 0  # ragged: blocks straddle boxes


def test_boxes_advective_term():
    w = small_boxes()
    h = make(w)
    A = to_np(h.advective_term(to_gpu(w["U0"])))
    ref = oracle_boxes(w, lambda U, p: osdc.A_of(U, p))
    e = rel_err_per_component(A, ref)
    print("boxes A max rel err", e.max())
    assert np.all(e <= 1e-11)


@pytest.mark.parametrize("precision,tol", [(0, TOL_FP64), (1, TOL_MIXED)])
def test_boxes_step(precision, tol):
    w = small_boxes()
    h = make(w, precision=precision)
    U = to_gpu(w["U0"])
    h.step(w["dt"], 2, U)
    ref = oracle_boxes(w, lambda Ub, p: osdc.run(Ub, w["dt"], 2, p))
    e = rel_err_per_component(to_np(U), ref)
    print(f"boxes step p{precision} max rel err {e.max():.3e}")
    assert np.all(e <= tol)
    st = h.stats()
    assert st["failed"] == 0 and st["solves"] == 2 * 2 * 4 * w["U0"].shape[1]


def test_lognormal_temperature_spreads_newton_counts():
    """The batched workload's per-zone temperatures spread the Newton counts."""
    w = small_boxes(nbox=24, choices=(4, 8), seed=5)
    h = make(w)
    U = to_gpu(w["U0"])
    h.step(w["dt"], 1, U)
    hist = np.array(h.stats()["hist"])
    used = np.nonzero(hist)[0]
    print("Newton histogram", dict(zip(used.tolist(), hist[used].tolist())))
    assert used.min() <= 2 and used.max() >= 7


def test_box_schedules_bitwise_identical():
    """Newton schedules and row-kernel tiles over the batched boxes (the
    tiles cut each box's z extent into chunks of its own) give the default
    bits, on boxes with spread Newton counts."""
    import torch
    w = small_boxes(nbox=12, choices=(4, 8, 12), seed=9)
    h = make(w)

    def one():
        U = to_gpu(w["U0"])
        h.stats_reset()
        h.step(w["dt"], 1, U)
        return U, h.stats()

    ref, sref = one()
    for sched in [(1, 0, 0, 0), (0, 2, 0, 0), (1, 3, 0, 4), (0, 0, 0, 2), (0, 0, 0, 16)]:
        h.set_schedule(*sched)
        U, s = one()
        assert bool(torch.equal(U, ref)), sched
        assert s == sref, sched
