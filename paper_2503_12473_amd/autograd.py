"""torch.autograd.Function around a fixed-step RK-OECDG run.

forward:  u(T) = run(u0) for nsteps steps of size dt (oecdg_run, dt fixed);
backward: dJ/du0 from dJ/du(T) with the hand-written discrete adjoint
          (oecdg_adjoint: checkpoints every `checkpoint_every` steps, segment
          recomputation, reverse stage kernels).
The time step is a fixed input, not differentiated.
"""
from __future__ import annotations

import torch


class OECDGRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, uC0, uD0, solver, nsteps, dt, checkpoint_every):
        uC, uD = uC0.detach().clone().contiguous(), uD0.detach().clone().contiguous()
        solver.run(uC, uD, nsteps=nsteps, dt_fixed=dt)
        ctx.save_for_backward(uC0.detach(), uD0.detach())
        ctx.solver, ctx.nsteps, ctx.dt, ctx.ckpt = solver, nsteps, dt, checkpoint_every
        return uC, uD

    @staticmethod
    def backward(ctx, gC, gD):
        uC0, uD0 = ctx.saved_tensors
        gC = torch.zeros_like(uC0) if gC is None else gC.contiguous()
        gD = torch.zeros_like(uD0) if gD is None else gD.contiguous()
        gC0, gD0 = ctx.solver.adjoint(uC0.contiguous(), uD0.contiguous(), ctx.nsteps, ctx.dt, gC, gD, ctx.ckpt)
        return gC0, gD0, None, None, None, None


def run_differentiable(solver, uC0, uD0, nsteps: int, dt: float, checkpoint_every: int = 20):
    """Differentiable fixed-step run: returns (uC(T), uD(T))."""
    return OECDGRun.apply(uC0, uD0, solver, nsteps, dt, checkpoint_every)
