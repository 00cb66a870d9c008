"""The allocation-free variant of the implicit reaction solve
(sdc_reaction_solve_noalloc) against sdc_reaction_solve, through the C ABI.

The variant runs the same kernels with the deferred-zone queue in the
library's fixed device array instead of a handle-owned allocation, so its
results must equal those of sdc_reaction_solve bit for bit (the solves are
zone-local).  Two calls in a row share the array: the second, on fewer zones,
must not see the first's queue contents.  The schedules cover a queue that
stays empty, zones deferred at an iteration cap, and every zone sent to the
pivoted dense path (pivot threshold above one).
"""
import ctypes

import numpy as np
import pytest

import sdc_inputs as si
from oracle import sdc as osdc
from tests.helpers import to_gpu, to_np

pytestmark = pytest.mark.gpu

SHAPE_BIG = (16, 16, 12)   # 3072 zones: 12 blocks of 256
SHAPE_SMALL = (10, 10, 10)  # 1000 zones: a ragged last block


def solve_inputs(w):
    prob = osdc.Problem.from_workload(w)
    rho, _, x0, _ = osdc.split_state(w["U0"], prob)
    g = si.rng(11)
    b = x0 * (1.0 + 0.05 * g.uniform(-1, 1, x0.shape))
    return rho, b, x0


def handle(shape, tau, cap):
    from paper_1910_12578_amd import SDC, config_from_workload
    w = si.workload("net3d", shape=shape)
    h = SDC(config_from_workload(w, pivot_threshold=tau), w["network"])
    h.set_schedule(0, cap)
    return w, h


def reference(h, dtm, rho, b, x0):
    x, R, it = h.reaction_solve(dtm, to_gpu(rho), to_gpu(b), to_gpu(x0))
    st = h.stats()
    h.stats_reset()
    return to_np(x), to_np(R), to_np(it), st


def noalloc(h, dtm, rho, b, x0):
    import torch
    nz = rho.size
    x = to_gpu(x0)
    R = torch.full_like(x, np.nan)
    it = torch.full((nz,), -7, dtype=torch.int32, device="cuda")
    h.reaction_solve_noalloc(dtm, to_gpu(rho), to_gpu(b), x, R, it)
    st = h.stats()
    h.stats_reset()
    return to_np(x), to_np(R), to_np(it), st


@pytest.mark.parametrize("tau,cap", [(0.1, 0), (0.1, 2), (2.0, 0)], ids=["fast", "capped", "dense"])
def test_noalloc_matches_reaction_solve(tau, cap):
    w, h = handle(SHAPE_BIG, tau, cap)
    ws, hs = handle(SHAPE_SMALL, tau, cap)
    try:
        dtm = 2.0 * w["dt"]
        rho, b, x0 = solve_inputs(w)
        print(f"[noalloc] tau={tau} cap={cap}: call 1 on {rho.size} zones", flush=True)
        ref = reference(h, dtm, rho, b, x0)
        got = noalloc(h, dtm, rho, b, x0)
        for r, g, name in zip(ref[:3], got[:3], ("x", "R", "iters")):
            assert np.array_equal(r, g), f"{name} differs (call 1)"
        assert ref[3] == got[3]
        if tau > 1.0:
            assert got[3]["fallbacks"] > 0  # the queue carried every zone
        if cap:
            assert max(ref[2]) > cap  # some zones went through the queue
        # call 2: fewer zones, other values, the array still holds call 1's queue
        rho2, b2, x02 = solve_inputs(ws)
        print(f"[noalloc] tau={tau} cap={cap}: call 2 on {rho2.size} zones", flush=True)
        ref2 = reference(hs, dtm, rho2, b2, x02)
        got2 = noalloc(h, dtm, rho2, b2, x02)
        for r, g, name in zip(ref2[:3], got2[:3], ("x", "R", "iters")):
            assert np.array_equal(r, g), f"{name} differs (call 2)"
        assert ref2[3] == got2[3]
        assert np.all(got2[2] > 0)
    finally:
        h.close()
        hs.close()


def test_noalloc_rejects_sizes_beyond_the_array():
    import torch
    from paper_1910_12578_amd import _binding
    w, h = handle(SHAPE_SMALL, 0.1, 0)
    try:
        t = torch.zeros(16, dtype=torch.float64, device="cuda")
        it = torch.zeros(16, dtype=torch.int32, device="cuda")
        L = _binding.lib()
        p = ctypes.c_void_p(t.data_ptr())
        # the size check precedes any launch: nothing is read through p
        rc = L.sdc_reaction_solve_noalloc(h._h, 1e-3, 10 ** 7, p, p, ctypes.c_void_p(t.data_ptr() + 64), p,
                                          ctypes.c_void_p(it.data_ptr()), None)
        assert rc == 1  # SDC_ERR_ARG
        assert b"exceeds the scratch array" in L.sdc_last_error(h._h)
        assert L.sdc_reaction_solve_noalloc(h._h, 1e-3, -1, p, p, p, p, p, None) == 1
        assert L.sdc_reaction_solve_noalloc(h._h, 1e-3, 0, None, None, None, None, None, None) == 0
    finally:
        h.close()
