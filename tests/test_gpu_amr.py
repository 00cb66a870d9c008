"""GPU parity of the two-level hierarchy (refined patches with subcycling,
the AMR extension that the paper names in Sec. 2 and Sec. 5) against the
oracle, and conservation on the composite grid.

The patches are padded boxes concatenated after each other; the whole padded
arrays (ghost zones included, which hold the last fill) and the coarse state
are compared with the oracle's two-level step at the FP64 bar (1e-8 in mixed
precision).
"""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import amr as oamr
from oracle import sdc as osdc
from tests.helpers import TOL_FP64, TOL_MIXED, rel_err_per_component, to_gpu, to_np

pytestmark = pytest.mark.gpu

CASES = {
    "chain1d": ((64,), [((10,), (12,)), ((40,), (9,))]),
    "net2d": ((40, 28), [((3, 2), (9, 7)), ((20, 14), (13, 11))]),
    "net3d": ((12, 10, 9), [((2, 3, 1), (5, 4, 6))]),
}


def setup(name, precision=0, **over):
    from paper_1910_12578_amd import AMR, config_from_workload
    shape, patches = CASES[name]
    w = si.workload(name, shape=shape)
    prob = osdc.Problem.from_workload(w, **{k: v for k, v in over.items() if k in ("slope", "alpha", "advection")})
    hier = oamr.Hierarchy(prob, [oamr.Patch(lo, ext) for lo, ext in patches])
    a = AMR(config_from_workload(w, precision=precision, **over), w["network"], patches)
    return w, hier, a


def concat(Ufs):
    return np.concatenate([U.reshape(U.shape[0], -1) for U in Ufs], axis=1)


def assert_close(got, ref, tol, what):
    e = rel_err_per_component(got, ref)
    print(f"{what}: max rel err per component {e.max():.3e}", flush=True)
    assert np.all(e <= tol), (what, e)


@pytest.mark.parametrize("name,nsteps,over", [("chain1d", 3, {}), ("net2d", 2, {}), ("net3d", 1, {}),
                                              ("net2d", 1, {"slope": 0, "alpha": 2.0}),
                                              ("net2d", 1, {"advection": 0})])
def test_two_level_step_matches_oracle(name, nsteps, over):
    import torch
    w, hier, a = setup(name, **over)
    nc = w["U0"].shape[0]
    Uc = to_gpu(w["U0"].reshape(nc, -1))
    Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
    a.fill_patches(Uc, Uf)
    Ufs = oamr.init_patches(w["U0"], hier)
    assert_close(to_np(Uf), concat(Ufs), 1e-14, f"patch fill {name}")
    print(f"[amr] {name} x{nsteps} {over}", flush=True)
    a.step(w["dt"], nsteps, Uc, Uf)
    U = w["U0"]
    for _ in range(nsteps):
        U, Ufs = oamr.amr_step(U, Ufs, w["dt"], hier)
    assert_close(to_np(Uc), U.reshape(nc, -1), TOL_FP64, f"coarse {name}")
    assert_close(to_np(Uf), concat(Ufs), TOL_FP64, f"patches {name}")
    for st in a.stats():
        assert st["failed"] == 0 and st["nonfinite"] == 0
    a.close()


def test_two_level_step_mixed_precision():
    import torch
    w, hier, a = setup("net2d", precision=1)
    nc = w["U0"].shape[0]
    Uc = to_gpu(w["U0"].reshape(nc, -1))
    Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
    a.fill_patches(Uc, Uf)
    Ufs = oamr.init_patches(w["U0"], hier)
    a.step(w["dt"], 2, Uc, Uf)
    U = w["U0"]
    for _ in range(2):
        U, Ufs = oamr.amr_step(U, Ufs, w["dt"], hier)
    assert_close(to_np(Uc), U.reshape(nc, -1), TOL_MIXED, "coarse mixed")
    assert_close(to_np(Uf), concat(Ufs), TOL_MIXED, "patches mixed")
    a.close()


def test_composite_conservation_on_a_large_grid():
    """256^2 coarse zones, three patches, 5 coarse steps: composite-grid mass,
    momentum and total energy (with the binding energy) constant to rounding."""
    import torch
    from paper_1910_12578_amd import AMR, config_from_workload
    w = si.workload("net2d", shape=(256, 256))
    patches = [((20, 30), (40, 50)), ((100, 120), (64, 64)), ((200, 10), (30, 100))]
    a = AMR(config_from_workload(w), w["network"], patches)
    nc = w["U0"].shape[0]
    Uc = to_gpu(w["U0"].reshape(nc, -1))
    Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
    a.fill_patches(Uc, Uf)
    prob = osdc.Problem.from_workload(w)
    hier = oamr.Hierarchy(prob, [oamr.Patch(lo, ext) for lo, ext in patches])

    def totals(f=lambda v: v):
        Ucn = f(to_np(Uc).reshape(w["U0"].shape))
        Ufn, off = f(to_np(Uf)), 0
        Ufs = []
        for p in hier.patches:
            shp = tuple(2 * e + 4 for e in p.ext)[::-1]
            n = int(np.prod(shp))
            Ufs.append(Ufn[:, off:off + n].reshape((nc,) + shp))
            off += n
        return oamr.composite_totals(Ucn, Ufs, hier)

    t0, scale = totals(), totals(np.abs)  # scale: the same sums of magnitudes
    a.step(w["dt"], 5, Uc, Uf)
    drift = np.abs(totals() - t0) / scale
    print("composite drift", drift)
    assert np.all(drift <= 1e-15), drift
    for st in a.stats():
        assert st["failed"] == 0 and st["nonfinite"] == 0
    a.close()


def test_hierarchy_rejects_bad_patches():
    from paper_1910_12578_amd import AMR, SDCError, config_from_workload
    w = si.workload("net2d", shape=(16, 16))
    with pytest.raises(SDCError, match="SDC_ERR_ARG"):
        AMR(config_from_workload(w), w["network"], [((2, 2), (4, 4)), ((7, 2), (3, 3))])  # one zone apart
    with pytest.raises(SDCError, match="SDC_ERR_ARG"):
        AMR(config_from_workload(w), w["network"], [((14, 2), (4, 4))])  # past the grid
    with pytest.raises(SDCError, match="SDC_ERR_ARG"):  # one zone apart across the periodic boundary
        AMR(config_from_workload(w), w["network"], [((1, 2), (4, 4)), ((8, 2), (8, 4))])
    with pytest.raises(SDCError, match="SDC_ERR_ARG"):  # meets itself across it
        AMR(config_from_workload(w), w["network"], [((0, 2), (15, 4))])
    AMR(config_from_workload(w), w["network"], [((2, 2), (4, 4)), ((8, 2), (6, 4))]).close()  # two zones apart both ways
    with pytest.raises(SDCError, match="SDC_ERR_UNSUPPORTED"):
        AMR(config_from_workload(w, space_order=4), w["network"], [((2, 2), (4, 4))])


def test_two_level_schedules_bitwise_identical():
    """The coarse level's Newton schedule, which the patches take over, only
    moves where iterations run: the two-level step gives the default bits."""
    import torch
    w, hier, a = setup("net3d")
    nc = w["U0"].shape[0]

    def one():
        Uc = to_gpu(w["U0"].reshape(nc, -1))
        Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
        a.fill_patches(Uc, Uf)
        a.step(w["dt"], 1, Uc, Uf)
        return Uc, Uf

    rc, rf = one()
    for sched in [(1, 0), (0, 2), (1, 3)]:
        a.set_schedule(*sched)
        Uc, Uf = one()
        assert bool(torch.equal(Uc, rc)) and bool(torch.equal(Uf, rf)), sched
    a.close()
