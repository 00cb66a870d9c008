"""torch.autograd.Function over SDC steps with the library's hand-written adjoint.

Forward runs `nsteps` SDC steps (the C ABI's sdc_step) and keeps the state
U^n at the start of every step as a checkpoint.  Backward walks the steps in
reverse, each through sdc_step_adjoint, which replays the step from its
checkpoint and differentiates every implicit reaction solve with the
implicit-function theorem at its converged root (paper Sec. 2, Eq. 2 for the
update being differentiated).  Gradients flow to the initial state and to the
rate parameters theta = (lnA_r, E_r).
"""
from __future__ import annotations

import numpy as np
import torch


class SDCSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, theta, solver, dt, nsteps):
        nr = solver.nreact
        th = theta.detach().to("cpu", torch.float64).numpy()
        solver.set_params(th[:nr], th[nr:])
        U = U0.detach().contiguous().clone()
        work = solver.alloc_nodes()
        ckpts = []
        for _ in range(int(nsteps)):
            ckpts.append(U.clone())
            solver.step(dt, 1, U, work)
        ctx.solver, ctx.dt, ctx.ckpts, ctx.theta = solver, float(dt), ckpts, th
        ctx.theta_device = theta.device
        return U

    @staticmethod
    def backward(ctx, Ubar):
        solver = ctx.solver
        nr = solver.nreact
        solver.set_params(ctx.theta[:nr], ctx.theta[nr:])
        thetabar = torch.zeros(2 * max(nr, 1), dtype=torch.float64, device="cuda")
        Ub = Ubar.detach().contiguous().to(torch.float64).clone()
        for U_n in reversed(ctx.ckpts):
            Ub, _ = solver.step_adjoint(ctx.dt, U_n, Ub, None, thetabar)
        return Ub, thetabar[:2 * nr].to(ctx.theta_device), None, None, None


def run_steps(solver, U0, theta, dt, nsteps):
    """U^N as a differentiable function of U0 and theta = (lnA, E)."""
    return SDCSteps.apply(U0, theta, solver, dt, nsteps)


def energy_released(U0, UN, q, dim, dV):
    """dV sum_z sum_i q_i [rho X_i(t0) - rho X_i(tN)] (total reaction energy)."""
    ns = q.numel()
    return dV * ((U0[2 + dim:2 + dim + ns] - UN[2 + dim:2 + dim + ns]) * q[:, None]).sum()


def theta_of(net):
    return torch.tensor(np.concatenate([net["lnA"], net["E"]]), dtype=torch.float64)
