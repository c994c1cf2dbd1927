"""Reverse-mode gradients of SSLBM runs for ``torch.autograd``.

``sslbm_run(rho0, theta, solver, nsteps, every)`` advances rho0 by nsteps
steps on the GPU with the parameters theta = (beta, alpha, gamma, phi,
d[0..4]) (Sec. II.A notation, physical diffusivities). Its backward pass is
the library's checkpointed reverse sweep: the forward stores the state every
``every`` steps, the backward recomputes each segment from its checkpoint and
runs the adjoint steps through it. Gradients flow to rho0 and theta.

``theta_from_sigma_mu`` builds theta from the (beta, sigma, gamma, mu) naming
with differentiable torch operations, so gradients with respect to those
rates follow by the chain rule.
"""
from __future__ import annotations

import torch

from .binding import GRAD_COUNT, Solver
from .inputs import Params

PARAM_NAMES = ("beta", "alpha", "gamma", "phi", "d_S", "d_E", "d_I", "d_R", "d_D")


def theta_of(p: Params) -> torch.Tensor:
    """theta (float64, CPU, 9) of a parameter set."""
    return torch.tensor([p.beta, p.alpha, p.gamma, p.phi, *p.d], dtype=torch.float64)


def params_of(theta: torch.Tensor, dx: float, dt: float) -> Params:
    v = [float(x) for x in theta.detach().cpu().tolist()]
    if len(v) != GRAD_COUNT:
        raise ValueError(f"theta must have {GRAD_COUNT} entries")
    return Params(beta=v[0], alpha=v[1], gamma=v[2], phi=v[3], d=tuple(v[4:]), dx=dx, dt=dt)


def theta_from_sigma_mu(beta, sigma, gamma, mu, d) -> torch.Tensor:
    """theta from (beta, sigma, gamma, mu): alpha = sigma, the paper's removal
    rate is gamma + mu and its fatality ratio mu / (gamma + mu)."""
    removal = gamma + mu
    return torch.stack([beta, sigma, removal, mu / removal, *d.unbind(0)])


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, theta, solver: Solver, nsteps: int, every: int):
        params = params_of(theta, solver.params.dx, solver.params.dt)
        solver.set_params(params)
        rho = rho0.detach().clone().contiguous()
        checkpoints = solver.run_checkpointed(rho, nsteps, every)
        ctx.solver, ctx.params, ctx.nsteps, ctx.every = solver, params, nsteps, every
        ctx.checkpoints = checkpoints
        ctx.theta_meta = (theta.dtype, theta.device)
        return rho

    @staticmethod
    def backward(ctx, grad_out):
        solver = ctx.solver
        solver.set_params(ctx.params)
        lam = grad_out.detach().to(solver.dtype).contiguous().clone()
        lam, grad = solver.adjoint_run(ctx.checkpoints, ctx.nsteps, ctx.every, lam)
        ctx.checkpoints = None
        dtype, device = ctx.theta_meta
        return lam, grad.to(dtype=dtype, device=device), None, None, None


def sslbm_run(rho0: torch.Tensor, theta: torch.Tensor, solver: Solver, nsteps: int,
              every: int = 100) -> torch.Tensor:
    """rho(T) after nsteps steps from rho0, differentiable in rho0 and theta."""
    return _Run.apply(rho0, theta, solver, int(nsteps), int(every))
