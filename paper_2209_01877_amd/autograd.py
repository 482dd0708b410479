"""torch.autograd front end of the residual VJP and the checkpointed SSP-RK3 adjoint.

All arithmetic runs in libtetdg: the forward residual and stages in the fused stage
kernel, the backward in the VJP kernel with its accumulating epilogue.
"""
from __future__ import annotations

import torch


class ResidualFn(torch.autograd.Function):
    """R(U) for an internal-layout state U; backward is (dR/dU)^T applied by the VJP kernel."""

    @staticmethod
    def forward(ctx, U, solver):
        ctx.solver = solver
        ctx.save_for_backward(U)
        return solver.residual(U.detach().contiguous())

    @staticmethod
    def backward(ctx, grad):
        (U,) = ctx.saved_tensors
        return ctx.solver.residual_vjp(U.detach().contiguous(), grad.contiguous()), None


def residual(solver, U: torch.Tensor) -> torch.Tensor:
    return ResidualFn.apply(U, solver)


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0, solver, dt, n_steps, checkpoint_every):
        U = U0.detach().clone()
        work = solver.new_work()
        ckpt = [U.clone()]
        done = 0
        while done < n_steps:
            k = min(checkpoint_every, n_steps - done)
            solver.rk_step(U, dt, k, work)
            done += k
            if done < n_steps:
                ckpt.append(U.clone())
        ctx.solver, ctx.dt, ctx.n, ctx.k = solver, dt, n_steps, checkpoint_every
        ctx.ckpt = ckpt
        return U

    @staticmethod
    def backward(ctx, grad):
        s, dt, n, k = ctx.solver, ctx.dt, ctx.n, ctx.k
        bar = grad.detach().contiguous().clone()
        starts = list(range(0, n, k))
        b2, b1, b0 = s.new_state(), s.new_state(), s.new_state()
        for seg in reversed(range(len(starts))):
            a = starts[seg]
            m = min(k, n - a)
            # recompute every stage state of this segment from its checkpoint
            stages = []
            U = ctx.ckpt[seg]
            for _ in range(m):
                U1 = s.rk_stage(U, None, s.new_state(), 0.0, dt)
                U2 = s.rk_stage(U1, U, s.new_state(), 0.75, dt)
                U3 = s.rk_stage(U2, U, s.new_state(), 1.0 / 3.0, dt)
                stages.append((U, U1, U2))
                U = U3
            for (U0s, U1s, U2s) in reversed(stages):
                s.residual_vjp_axpy(U2s, bar, 2.0 / 3.0 * dt, [(2.0 / 3.0, bar)], b2)
                s.residual_vjp_axpy(U1s, b2, 0.25 * dt, [(0.25, b2)], b1)
                s.residual_vjp_axpy(U0s, b1, dt, [(1.0, b1), (0.75, b2), (1.0 / 3.0, bar)], b0)
                bar, b0 = b0, bar
        return bar, None, None, None, None


def rk_trajectory(solver, U0: torch.Tensor, dt: float, n_steps: int, checkpoint_every: int = 10) -> torch.Tensor:
    """U_n after n SSP-RK3 steps; differentiable w.r.t. U0 through the discrete adjoint,
    with the forward states stored every `checkpoint_every` steps and the stage states of
    one segment recomputed during the backward pass."""
    return _Trajectory.apply(U0, solver, float(dt), int(n_steps), int(checkpoint_every))
