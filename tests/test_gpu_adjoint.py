"""Adjoint of the SDC step (gradients of integrated energy release with respect
to the rate parameters and the initial state) against finite differences of
the GPU forward and against the oracle's complex-step gradient."""
import numpy as np
import pytest

import sdc_inputs as si
from oracle import adjoint as oadj
from oracle import sdc as osdc
from tests.helpers import to_gpu

pytestmark = pytest.mark.gpu


def setup(shape=(24, 20), **over):
    import torch
    from paper_1910_12578_amd import SDC, config_from_workload
    w = si.workload("adjoint2d", shape=shape)
    h = SDC(config_from_workload(w, **over), w["network"])
    q = torch.tensor(w["network"]["q"], dtype=torch.float64, device="cuda")
    return w, h, q


def objective(h, w, q, U0, theta, nsteps):
    from paper_1910_12578_amd.autograd import energy_released, run_steps
    UN = run_steps(h, U0, theta, w["dt"], nsteps)
    return energy_released(U0, UN, q, w["dim"], float(np.prod(w["dx"])))


def test_parameter_gradient_matches_finite_differences():
    import torch
    from paper_1910_12578_amd.autograd import theta_of
    w, h, q = setup()
    nsteps = 3
    nc = w["U0"].shape[0]
    U0 = to_gpu(w["U0"].reshape(nc, -1))
    theta = theta_of(w["network"]).requires_grad_(True)
    J = objective(h, w, q, U0, theta, nsteps)
    J.backward()
    g = theta.grad.numpy()
    nr = w["network"]["nreact"]
    fd = np.zeros_like(g)
    for p in range(2 * nr):
        hstep = 1e-4 if p < nr else 1e-4 * w["network"]["E"][p - nr]
        with torch.no_grad():
            tp, tm = theta.detach().clone(), theta.detach().clone()
            tp[p] += hstep
            tm[p] -= hstep
            fd[p] = (objective(h, w, q, U0, tp, nsteps).item() - objective(h, w, q, U0, tm, nsteps).item()) / (2 * hstep)
    scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    err = np.abs(g - fd) / scale
    print("adjoint vs FD: max scaled error", err.max(), "max |g|", np.abs(fd).max())
    assert np.all(err <= 1e-6), (g, fd)


@pytest.mark.parametrize("n_nodes", [4, 5])
def test_parameter_gradient_at_four_and_five_nodes(n_nodes):
    """Regression: the adjoint at 4 and 5 Gauss-Lobatto nodes, where the first
    zeroing launch of the reverse pass takes 3 (M + 1) = 12 and 15 arrays
    (every node's U, A and R adjoints), against central differences of the
    GPU forward on the parameters with the largest gradients."""
    import torch
    from paper_1910_12578_amd.autograd import theta_of
    print(f"adjoint at {n_nodes} nodes", flush=True)
    w, h, q = setup(shape=(12, 10), n_nodes=n_nodes, n_iters=3)
    nsteps = 2
    nc = w["U0"].shape[0]
    U0 = to_gpu(w["U0"].reshape(nc, -1))
    theta = theta_of(w["network"]).requires_grad_(True)
    J = objective(h, w, q, U0, theta, nsteps)
    J.backward()
    g = theta.grad.numpy()
    nr = w["network"]["nreact"]
    picks = np.argsort(-np.abs(g))[:6]
    fd = np.zeros(picks.size)
    for i, p in enumerate(picks):
        hstep = 1e-4 if p < nr else 1e-4 * w["network"]["E"][p - nr]
        with torch.no_grad():
            tp, tm = theta.detach().clone(), theta.detach().clone()
            tp[p] += hstep
            tm[p] -= hstep
            fd[i] = (objective(h, w, q, U0, tp, nsteps).item() - objective(h, w, q, U0, tm, nsteps).item()) / (2 * hstep)
    err = np.abs(g[picks] - fd) / np.abs(fd)
    print(f"{n_nodes} nodes: adjoint vs FD max relative error {err.max():.2e}")
    assert np.all(err <= 1e-6), (g[picks], fd)


def test_parameter_gradient_matches_oracle_complex_step():
    import torch
    from paper_1910_12578_amd.autograd import theta_of
    w, h, q = setup(shape=(16, 16))
    nsteps = 3
    nc = w["U0"].shape[0]
    theta = theta_of(w["network"]).requires_grad_(True)
    J = objective(h, w, q, to_gpu(w["U0"].reshape(nc, -1)), theta, nsteps)
    J.backward()
    g = theta.grad.numpy()
    prob = osdc.Problem.from_workload(w)
    g_lnA, g_E = oadj.energy_gradient(w["U0"], w["dt"], nsteps, prob)
    ref = np.concatenate([g_lnA, g_E])
    err = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    print("adjoint vs oracle complex step: max scaled error", err.max())
    assert np.all(err <= 1e-8), (g, ref)


def test_parameter_gradient_64sq_20_steps_matches_oracle():
    """The adjoint at 64^2 zones over 20 steps against the oracle's
    complex-step gradient of the same run (stored by
    tests/golden/make_adjoint_gradient.py, which calls only the oracle)."""
    from paper_1910_12578_amd.autograd import theta_of
    from tests import golden
    ref = golden.read("adjoint_gradient_64sq_20steps.txt")
    ref = np.concatenate([ref["dlnA"], ref["dE"]])
    w, h, q = setup(shape=(64, 64))
    nc = w["U0"].shape[0]
    theta = theta_of(w["network"]).requires_grad_(True)
    J = objective(h, w, q, to_gpu(w["U0"].reshape(nc, -1)), theta, 20)
    J.backward()
    g = theta.grad.numpy()
    err = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    print("adjoint 64^2 x 20 vs oracle complex step: max scaled error", err.max())
    assert np.all(err <= 1e-8), (g, ref)


def test_state_gradient_directional_derivative():
    import torch
    from paper_1910_12578_amd.autograd import theta_of
    w, h, q = setup(shape=(16, 12))
    nsteps = 2
    nc = w["U0"].shape[0]
    U0 = to_gpu(w["U0"].reshape(nc, -1)).requires_grad_(True)
    theta = theta_of(w["network"])
    J = objective(h, w, q, U0, theta, nsteps)
    J.backward()
    G = U0.grad.detach()
    g = si.rng(3)
    for trial in range(3):
        v = torch.from_numpy(g.standard_normal(U0.shape) * np.abs(w["U0"].reshape(nc, -1)) * 1e-3).cuda()
        eps = 1e-3
        with torch.no_grad():
            Jp = objective(h, w, q, U0.detach() + eps * v, theta, nsteps).item()
            Jm = objective(h, w, q, U0.detach() - eps * v, theta, nsteps).item()
        fd = (Jp - Jm) / (2 * eps)
        ad = float((G * v).sum())
        print(f"directional: adjoint {ad:.10e} FD {fd:.10e}")
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-18


def test_adjoint_needs_smooth_mode():
    import torch
    from paper_1910_12578_amd import SDCError
    w, h, q = setup(slope=1)
    nc = w["U0"].shape[0]
    U = to_gpu(w["U0"].reshape(nc, -1))
    with pytest.raises(SDCError):
        h.step_adjoint(w["dt"], U, torch.zeros_like(U))


def test_adjoint_is_deterministic():
    import torch
    w, h, q = setup(shape=(16, 16))
    nc = w["U0"].shape[0]
    U = to_gpu(w["U0"].reshape(nc, -1))
    seed = torch.zeros_like(U)
    seed[2 + w["dim"]:] = -1.0
    a, ta = h.step_adjoint(w["dt"], U, seed)
    b, tb = h.step_adjoint(w["dt"], U, seed)
    assert bool((a == b).all()) and bool((ta == tb).all())
