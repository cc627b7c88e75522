"""Differentiable real-time SS-CN propagation (torch.autograd.Function).

``propagate(psi0, omega, problem)`` returns the state after ``problem.steps``
real-time steps, where step n uses Rabi strength ``omega[n // steps_per_seg]``
(piecewise-constant control).  Its backward pass gives the gradients with
respect to the initial state and to every Omega segment, in torch's
convention for complex tensors (dL/dRe + i dL/dIm).

Memory follows the checkpointing scheme: the forward pass keeps one state
every ``checkpoint`` steps (default ceil(sqrt(steps))); the backward pass
walks the segments from the last to the first, recomputes the segment's
step inputs from its checkpoint into a segment buffer, and runs the adjoint
steps over them (CN_y^H, CN_x^H, SO^H and the transposed HERM o CALCNU
Jacobian, all in the HIP kernels).  The recomputation of segment s - 1 does
not depend on the adjoint steps of segment s, so it runs beside them: on a
second grid object bound to a stream of its own, into the other of two
segment buffers, ordered by events (the adjoint of a segment waits for its
recomputation; a recomputation waits until the adjoint steps that last read
its buffer are done).  Every kernel does the same arithmetic in the same
order as with one stream, so the gradients are the same bits.
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
        ctx.omega_list = omega.detach().cpu().tolist()
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
        main = torch.cuda.current_stream(lam.device)
        side = torch.cuda.Stream(device=lam.device)  # default priority
        nbuf = 2 if len(ctx.checkpoints) > 1 else 1
        segs = [torch.empty((C,) + tuple(shape), dtype=lam.dtype, device=lam.device) for _ in range(nbuf)]
        side.wait_stream(main)  # the checkpoints, lam and the buffers are ready
        # the grid object of the recomputation: same parameters and schedule,
        # its launches on `side`; its bound state is never used (step_real_seq
        # reads src and writes dst)
        g2 = api.Grid(ctx.checkpoints[0], prob.dx, prob.dy, stream=side)
        g2.set_params(g.p)
        g2.set_omega_schedule(ctx.omega_list, prob.steps_per_seg)
        freed = [None] * nbuf  # event: the adjoint steps that last read buffer b are done

        def recompute(s):
            """Segment s's step inputs into buffer s % nbuf, on `side`; returns
            the event that marks them written."""
            seg = segs[s % nbuf]
            n0 = s * C
            n = min(C, prob.steps - n0)
            with torch.cuda.stream(side):
                if freed[s % nbuf] is not None:
                    side.wait_event(freed[s % nbuf])
                seg[0].copy_(ctx.checkpoints[s])
                if n > 1:
                    g2.step_index = n0
                    g2.step_real_seq(seg[0], seg[1:n], n - 1)
                done = torch.cuda.Event()
                done.record(side)
            return done

        last = len(ctx.checkpoints) - 1
        ready = recompute(last)
        for s in reversed(range(len(ctx.checkpoints))):
            nxt = recompute(s - 1) if s > 0 else None
            n0 = s * C
            n = min(C, prob.steps - n0)
            main.wait_event(ready)
            g.step_index = n0 + n
            g.step_real_adjoint(segs[s % nbuf][:n], lam, n)
            freed[s % nbuf] = torch.cuda.Event()
            freed[s % nbuf].record(main)
            ready = nxt
        main.wait_stream(side)
        for seg in segs:
            seg.record_stream(side)
        g2.close()
        (omega,) = ctx.saved_tensors
        # the gradient lives where (and in the dtype that) the caller's Omega does
        domega = torch.tensor(g.omega_grad(reset=True), dtype=omega.dtype, device=omega.device)
        ctx.checkpoints = None
        return lam, domega, None


def propagate(psi0: torch.Tensor, omega: torch.Tensor, prob: RealTimeProblem) -> torch.Tensor:
    """State after prob.steps real-time steps (differentiable in psi0, omega)."""
    return _Propagate.apply(psi0, omega, prob)
