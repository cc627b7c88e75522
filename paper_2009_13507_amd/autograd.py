"""Differentiable real-time SS-CN propagation (torch.autograd.Function).

``propagate(psi0, omega, problem)`` returns the state after ``problem.steps``
real-time steps, where step n uses Rabi strength ``omega[n // steps_per_seg]``
(piecewise-constant control).  Its backward pass gives the gradients with
respect to the initial state and to every Omega segment, in torch's
convention for complex tensors (dL/dRe + i dL/dIm).

Memory follows the checkpointing scheme: the forward pass keeps one state
every ``checkpoint`` steps (default ceil(sqrt(steps))); the backward pass
walks the segments from the last to the first, recomputes the segment's
step inputs from its checkpoint into one segment buffer, and runs the
adjoint steps over them (CN_y^H, CN_x^H, SO^H and the transposed
HERM o CALCNU Jacobian, all in the HIP kernels).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

from . import api


@dataclass
class RealTimeProblem:
    dx: float
    dy: float
    dt: float
    steps: int
    steps_per_seg: int
    c0: float = 0.0
    c2: float = 0.0
    gamma: float = 0.0
    so: int = api.SO_PX_SX
    kappa: float = 1.0
    checkpoint: int | None = None

    def interval(self) -> int:
        return self.checkpoint or max(1, math.ceil(math.sqrt(self.steps)))


class _Propagate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0: torch.Tensor, omega: torch.Tensor, prob: RealTimeProblem):
        work = psi0.detach().clone().contiguous()
        g = api.Grid(work, prob.dx, prob.dy)
        g.set_params(c0=prob.c0, c2=prob.c2, gamma=prob.gamma, omega=0.0, dt=prob.dt, so=prob.so,
                     kappa=prob.kappa)
        g.set_omega_schedule(omega.detach().cpu().tolist(), prob.steps_per_seg)
        g.step_index = 0
        C = prob.interval()
        checkpoints = []
        done = 0
        while done < prob.steps:
            checkpoints.append(work.clone())
            n = min(C, prob.steps - done)
            g.step_real(n)
            done += n
        ctx.prob = prob
        ctx.grid = g
        ctx.save_for_backward(omega)
        ctx.checkpoints = checkpoints
        return work.clone()

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        prob = ctx.prob
        g = ctx.grid
        C = prob.interval()
        lam = grad_out.detach().clone().contiguous()
        g.omega_grad(reset=True)  # clear the accumulators
        shape = lam.shape
        seg = torch.empty((C,) + tuple(shape), dtype=lam.dtype, device=lam.device)
        for s in reversed(range(len(ctx.checkpoints))):
            n0 = s * C
            n = min(C, prob.steps - n0)
            seg[0].copy_(ctx.checkpoints[s])
            if n > 1:
                g.step_index = n0
                g.step_real_seq(seg[0], seg[1:n], n - 1)
            g.step_index = n0 + n
            g.step_real_adjoint(seg[:n], lam, n)
        (omega,) = ctx.saved_tensors
        # the gradient lives where (and in the dtype that) the caller's Omega does
        domega = torch.tensor(g.omega_grad(reset=True), dtype=omega.dtype, device=omega.device)
        ctx.checkpoints = None
        return lam, domega, None


def propagate(psi0: torch.Tensor, omega: torch.Tensor, prob: RealTimeProblem) -> torch.Tensor:
    """State after prob.steps real-time steps (differentiable in psi0, omega)."""
    return _Propagate.apply(psi0, omega, prob)
