"""Differentiable wrappers around the C ABI (torch.autograd.Function).

Every forward and backward step runs in the library's HIP kernels; torch only
chains the pieces:

* ``SetState``     (rho, v, P) -> U   (dg_set_state / dg_set_state_vjp)
* ``Trajectory``   U0 -> U after nsteps SSP-RK3 steps, checkpointing U every
                   ``k`` steps in the forward pass; the backward pass recomputes
                   each segment from its checkpoint with taped steps
                   (dg_ssprk3_run_tape) and runs the step adjoints in reverse
                   (dg_ssprk3_run_vjp_tape).  Memory: nsteps/k states of
                   checkpoints plus k tapes of 6 states.
* ``VY2``          U -> J = int v_y^2 dA (dg_objective_vy2 with its gradient)
"""
from __future__ import annotations

import torch


class SetState(torch.autograd.Function):
    @staticmethod
    def forward(ctx, src, solver):
        src = src.detach().contiguous()
        ctx.solver = solver
        ctx.save_for_backward(src)
        return solver.set_state(src)

    @staticmethod
    def backward(ctx, lamU):
        (src,) = ctx.saved_tensors
        return ctx.solver.set_state_vjp(src, lamU.contiguous()), None


class Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, nsteps: int, dt: float, k: int):
        U = U0.detach().contiguous().clone()
        ckpts = []
        s = 0
        while s < nsteps:
            ckpts.append(U.clone())
            n = min(k, nsteps - s)
            solver.run(U, dt, n)
            s += n
        ctx.solver, ctx.nsteps, ctx.dt, ctx.k, ctx.ckpts = solver, nsteps, dt, k, ckpts
        return U

    @staticmethod
    def backward(ctx, lam):
        solver, nsteps, dt, k = ctx.solver, ctx.nsteps, ctx.dt, ctx.k
        lam = lam.contiguous().clone()
        tapes = torch.empty((min(k, nsteps), solver.tape_numel), dtype=torch.float64, device=lam.device)
        for seg in reversed(range(len(ctx.ckpts))):
            s0 = seg * k
            n = min(k, nsteps - s0)
            U = ctx.ckpts[seg].clone()
            solver.run_tape(U, dt, n, tapes)
            solver.run_vjp_tape(tapes, dt, n, lam)
        ctx.ckpts = None
        return lam, None, None, None, None


class VY2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, solver):
        J, g = solver.objective_vy2(U.detach().contiguous(), grad=True)
        ctx.save_for_backward(g)
        return torch.tensor(J, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        return g * gJ, None


def trajectory(solver, U0, nsteps: int, dt: float, k: int = 20):
    return Trajectory.apply(U0, solver, nsteps, dt, k)


def vy2_after(solver, src, nsteps: int, dt: float, k: int = 20):
    """J(src) = int v_y^2 dA after nsteps steps from the primitive initial data src."""
    return VY2.apply(trajectory(solver, SetState.apply(src, solver), nsteps, dt, k), solver)
