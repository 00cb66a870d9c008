"""Parity at the full benchmark sizes (paper Sec. 2, Eq. 1 and Eq. 2).

The oracle cannot step a whole 256^3 grid in seconds, so it checks sampled
outputs: one SDC step moves information at most 2 zones per evaluation of
A(U), and a 3-node, K = 4 step chains 8 of them behind U^{n+1}, so the new
state of a zone depends on U^n within 16 zones.  The oracle steps a periodic
window of half-width W > 16 cut (with the grid's periodic wrap) around a
sample point; zones within W - 16 of the centre see no trace of the window's
own wrap and must match the full-grid GPU step.  Properties that hold at any
size (conservation of mass, momentum and total energy) are checked on the
whole grid.  The batched boxes are checked box by box on the smallest boxes,
and the adjoint against finite differences of the full 256^2, 20-step run.
"""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import sdc as osdc
from tests.helpers import TOL_FP64, TOL_MIXED, to_gpu

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

RADIUS = 16  # dependency radius of one 3-node, K = 4 step


def window(U0, centre, W):
    """Periodic window of half-width W around `centre` (x, y[, z]) of U0
    [comp, (z,) y, x], with the indices it takes."""
    idx = [np.arange(c - W, c + W + 1) % n for c, n in zip(centre, U0.shape[:0:-1])]
    if len(idx) == 3:
        win = U0[:, idx[2][:, None, None], idx[1][None, :, None], idx[0][None, None, :]]
    else:
        win = U0[:, idx[1][:, None], idx[0][None, :]]
    return np.ascontiguousarray(win), idx


def core_zones(idx, W, shape):
    """Linear zone indices (x fastest) and window positions of the core."""
    r = W - RADIUS
    sl = slice(W - r, W + r + 1)
    if len(idx) == 3:
        zz, yy, xx = np.meshgrid(idx[2][sl], idx[1][sl], idx[0][sl], indexing="ij")
        lin = xx + shape[0] * (yy + shape[1] * zz)
    else:
        yy, xx = np.meshgrid(idx[1][sl], idx[0][sl], indexing="ij")
        lin = xx + shape[0] * yy
    return lin.ravel(), sl


def gpu_step(w, precision, nsteps=1, schedule=None):
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    nc = w["U0"].shape[0]
    with SDC(config_from_workload(w, precision=precision), w["network"]) as h:
        if schedule is not None:
            h.set_schedule(*schedule)
        U = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
        h.step(w["dt"], nsteps, U)
        torch.cuda.synchronize()
        st = h.stats()
    return U, st


def conserved_totals(U, dim, q):
    """Sums of rho, rho u_d and of the total energy including the binding
    energy, rho E + sum_i q_i rho X_i (reactions move energy between the two:
    R_e + q . R_X = 0), over all zones (float64, on the GPU)."""
    ns = len(q)
    qt = q.to(U.device)[:, None]
    E_tot = U[1 + dim] + (qt * U[2 + dim:2 + dim + ns]).sum(dim=0)
    return np.array([float(U[c].sum()) for c in range(1 + dim)] + [float(E_tot.sum())])


@pytest.fixture(scope="module")
def net3d_full():
    w = si.workload("net3d")
    W = RADIUS + 2
    centres = [(100, 7, 250), (0, 255, 128)]  # interior, and across the periodic faces
    refs = []
    for c in centres:
        win, idx = window(w["U0"], c, W)
        prob = osdc.Problem.from_workload(dict(w, shape=(2 * W + 1,) * 3))
        out = osdc.run(win, w["dt"], 1, prob)
        lin, sl = core_zones(idx, W, w["shape"])
        refs.append((lin, out[:, sl, sl, sl].reshape(out.shape[0], -1)))
    return w, refs


# the schedules the autotuner picks at 256^3 (two-wave FP64 transitions, the
# compiler's budget in mixed precision, 128-plane advection tiles, which cut
# the z extent into two chunks) and the default one
@pytest.mark.parametrize("precision,tol,schedule", [(0, TOL_FP64, (1, 0, 0, 128)), (1, TOL_MIXED, (0, 0, 0, 128)),
                                                    (0, TOL_FP64, (0, 0, 0, 0))])
def test_net3d_256cubed_sampled_windows(net3d_full, precision, tol, schedule):
    """256^3 x 13 species, one step in the schedule bench.py times, against
    the oracle on two 37^3 windows (core 5^3 each), and global conservation."""
    import torch
    w, refs = net3d_full
    U, st = gpu_step(w, precision, schedule=schedule)
    assert st["failed"] == 0 and st["nonfinite"] == 0
    for lin, ref in refs:
        got = U[:, torch.from_numpy(lin).to("cuda")].cpu().numpy()
        err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
        print(f"precision {precision}: core max rel err per component {err.max():.3e}")
        assert np.all(err <= tol), err
    nc = w["U0"].shape[0]
    q = torch.tensor(w["network"]["q"], dtype=torch.float64)
    U0g = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
    before, after = conserved_totals(U0g, 3, q), conserved_totals(U, 3, q)
    scale = np.array([float(U0g[c].abs().sum()) for c in range(4)] + [float(U0g[4].abs().sum())])
    drift = np.abs(after - before) / scale
    print("conservation drift (rho, rho u, rho E + q.rho X):", drift)
    assert np.all(drift <= 1e-13), drift


def test_net3d_256cubed_fourth_order_sampled_windows():
    """The fourth-order leg at its full size (256^3 x 13 species, one step in
    the tuned schedule the bench times) against the oracle's fourth-order
    step on two 41^3 windows (core 9^3 each), and global conservation.  A
    fourth-order evaluation of A reaches 2 zones along a direction (face
    averages over 4 zones) and 1 across it, and the centre/average
    conversions 1 zone, so one step stays within the same 16-zone radius
    (a single-zone perturbation moves 8 zones in one step of the oracle)."""
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    w = dict(si.workload("net3d"), space_order=4)
    W = RADIUS + 4
    centres = [(200, 31, 5), (255, 0, 128)]
    refs = []
    for c in centres:
        win, idx = window(w["U0"], c, W)
        prob = osdc.Problem.from_workload(dict(w, shape=(2 * W + 1,) * 3))
        out = osdc.run(win, w["dt"], 1, prob)
        lin, sl = core_zones(idx, W, w["shape"])
        refs.append((lin, out[:, sl, sl, sl].reshape(out.shape[0], -1)))
    nc = w["U0"].shape[0]
    with SDC(config_from_workload(w, autotune=1), w["network"]) as h:
        U0g = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
        U = U0g.clone()
        h.step(w["dt"], 1, U)
        torch.cuda.synchronize()
        st = h.stats()
    assert st["failed"] == 0 and st["nonfinite"] == 0
    for lin, ref in refs:
        got = U[:, torch.from_numpy(lin).to("cuda")].cpu().numpy()
        err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
        print(f"fourth order: core max rel err per component {err.max():.3e}")
        assert np.all(err <= TOL_FP64), err
    q = torch.tensor(w["network"]["q"], dtype=torch.float64)
    before, after = conserved_totals(U0g, 3, q), conserved_totals(U, 3, q)
    scale = np.array([float(U0g[c].abs().sum()) for c in range(4)] + [float(U0g[4].abs().sum())])
    drift = np.abs(after - before) / scale
    print("conservation drift (rho, rho u, rho E + q.rho X):", drift)
    assert np.all(drift <= 1e-13), drift


def test_refined_patches_at_the_bench_size_conserve():
    """The refined-patch leg at its full size: the 256^3 coarse level with the
    bench's two patches refined by 2 (about 4.6e6 fine zones), two coarse
    steps with subcycling in the tuned schedule; the composite-grid mass,
    momentum and total energy stay constant to rounding (the refluxing), and
    every solve converges."""
    import torch
    from oracle import amr as oamr
    from paper_1910_12578_amd import AMR, config_from_workload
    w = si.workload("net3d")
    patches = [((32, 40, 48), (62, 64, 64)), ((150, 130, 120), (62, 64, 80))]
    nc = w["U0"].shape[0]
    a = AMR(config_from_workload(w, autotune=1), w["network"], patches)
    try:
        Uc = torch.from_numpy(w["U0"].reshape(nc, -1)).to("cuda")
        Uf = torch.empty((nc, a.zf), dtype=torch.float64, device="cuda")
        a.fill_patches(Uc, Uf)
        hier = oamr.Hierarchy(osdc.Problem.from_workload(w), [oamr.Patch(lo, ext) for lo, ext in patches])

        def totals(f=lambda v: v):
            Ucn = f(Uc.cpu().numpy().reshape(w["U0"].shape))
            Ufn, off, Ufs = f(Uf.cpu().numpy()), 0, []
            for p in hier.patches:
                shp = tuple(2 * e + 4 for e in p.ext)[::-1]
                n = int(np.prod(shp))
                Ufs.append(Ufn[:, off:off + n].reshape((nc,) + shp))
                off += n
            return oamr.composite_totals(Ucn, Ufs, hier)

        t0, scale = totals(), totals(np.abs)
        a.step(w["dt"], 2, Uc, Uf)
        torch.cuda.synchronize()
        drift = np.abs(totals() - t0) / scale
        print("composite drift", drift)
        assert np.all(drift <= 1e-15), drift
        for st in a.stats():
            assert st["failed"] == 0 and st["nonfinite"] == 0
    finally:
        a.close()


def test_net2d_512sq_sampled_windows():
    """512^2 x 7 species (zone-per-thread advective kernel), FP64 and mixed,
    against the oracle on four 49^2 windows (core 17^2 each)."""
    import torch
    w = si.workload("net2d")
    W = RADIUS + 8
    centres = [(3, 500), (256, 256), (511, 0), (77, 301)]
    refs = []
    for c in centres:
        win, idx = window(w["U0"], c, W)
        prob = osdc.Problem.from_workload(dict(w, shape=(2 * W + 1,) * 2))
        out = osdc.run(win, w["dt"], 1, prob)
        lin, sl = core_zones(idx, W, w["shape"])
        refs.append((lin, out[:, sl, sl].reshape(out.shape[0], -1)))
    for precision, tol in ((0, TOL_FP64), (1, TOL_MIXED)):
        U, st = gpu_step(w, precision)
        assert st["failed"] == 0
        for lin, ref in refs:
            got = U[:, torch.from_numpy(lin).to("cuda")].cpu().numpy()
            err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
            assert np.all(err <= tol), (precision, err)


def test_boxes_4096_full_size():
    """The 4096-box workload (1.09e8 zones) in one step: the smallest boxes
    against the oracle box by box, every box's mass, momentum and total energy
    conserved."""
    import torch
    w = si.boxes_workload()
    ext, off = np.asarray(w["box_n"]), np.asarray(w["box_off"])
    U, st = gpu_step(w, 0)
    assert st["failed"] == 0 and st["nonfinite"] == 0
    small = np.argsort(np.prod(ext, axis=1), kind="stable")[:3]
    for b in small:
        nx, ny, nz = ext[b]
        U0b = w["U0"][:, off[b]:off[b + 1]].reshape(-1, nz, ny, nx)
        prob = osdc.Problem.from_workload(dict(w, shape=(nx, ny, nz), box_n=None, box_off=None))
        ref = osdc.run(U0b, w["dt"], 1, prob).reshape(U0b.shape[0], -1)
        got = U[:, off[b]:off[b + 1]].cpu().numpy()
        err = np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)
        print(f"box {b} {tuple(ext[b])}: max rel err per component {err.max():.3e}")
        assert np.all(err <= TOL_FP64), err
    # conservation per box: segment sums of rho, rho u and rho E + q . rho X
    seg = torch.repeat_interleave(torch.arange(len(ext), device="cuda"),
                                  torch.from_numpy(np.diff(off)).to("cuda"))
    qt = torch.tensor(w["network"]["q"], dtype=torch.float64, device="cuda")[:, None]
    ns = qt.shape[0]

    def totals(V):
        rows = [V[c] for c in range(4)] + [V[4] + (qt * V[5:5 + ns]).sum(dim=0)]
        return [torch.zeros(len(ext), dtype=torch.float64, device="cuda").index_add_(0, seg, r) for r in rows], \
               [torch.zeros(len(ext), dtype=torch.float64, device="cuda").index_add_(0, seg, r.abs()) for r in rows]

    U0g = torch.from_numpy(w["U0"]).to("cuda")
    (s0, a0), (s1, _) = totals(U0g), totals(U)
    for c in range(5):
        drift = float(((s1[c] - s0[c]).abs() / a0[c]).max())
        assert drift <= 1e-12, (c, drift)


def test_adjoint_256sq_20_steps_matches_finite_differences():
    """Gradient of the energy released over 20 steps of the 256^2 smooth
    workload with respect to (lnA_r, E_r) against central differences of the
    same GPU forward runs (h = 1e-4 in lnA, 1e-4 E in E)."""
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    from paper_1910_12578_amd.autograd import energy_released, run_steps, theta_of
    w = si.workload("adjoint2d")
    nsteps = 20
    nc = w["U0"].shape[0]
    U0 = to_gpu(w["U0"].reshape(nc, -1))
    q = torch.tensor(w["network"]["q"], dtype=torch.float64, device="cuda")
    dV = float(np.prod(w["dx"]))
    with SDC(config_from_workload(w), w["network"]) as h:
        def J(theta):
            return energy_released(U0, run_steps(h, U0, theta, w["dt"], nsteps), q, w["dim"], dV)

        theta = theta_of(w["network"]).requires_grad_(True)
        J(theta).backward()
        g = theta.grad.numpy()
        nr = w["network"]["nreact"]
        fd = np.zeros_like(g)
        with torch.no_grad():
            for p in range(2 * nr):
                hs = 1e-4 if p < nr else 1e-4 * w["network"]["E"][p - nr]
                tp, tm = theta.detach().clone(), theta.detach().clone()
                tp[p] += hs
                tm[p] -= hs
                fd[p] = (J(tp).item() - J(tm).item()) / (2 * hs)
    scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    err = np.abs(g - fd) / scale
    print("full-size adjoint vs FD: max scaled error", err.max())
    assert np.all(err <= 1e-6), err
