"""Oracle adjoint: reverse-mode automatic differentiation through the oracle residual.

The paper has no adjoint.  The vector-Jacobian product (dR/dU)^T W is obtained
by torch autograd through the plain residual of oracle.dg, and the discrete
adjoint of several SSP-RK3 steps by autograd through the steps (recomputed from
checkpoints, which only bounds memory and does not change the result).
"""
from __future__ import annotations

import torch


def residual_vjp(dg, U: torch.Tensor, W: torch.Tensor) -> torch.Tensor:
    Ur = U.detach().clone().requires_grad_(True)
    R = dg.residual(Ur)
    (g,) = torch.autograd.grad(R, Ur, W)
    return g


def trajectory_vjp(dg, U0: torch.Tensor, dt: float, n_steps: int, W: torch.Tensor,
                   checkpoint_every: int = 10) -> torch.Tensor:
    """d<W, U_n>/dU_0 for n SSP-RK3 steps, segment by segment from stored checkpoints."""
    ckpt = [U0.detach().clone()]
    U = U0.detach()
    for s in range(n_steps):
        U = dg.rk3_step(U, dt)
        if (s + 1) % checkpoint_every == 0 and s + 1 < n_steps:
            ckpt.append(U.detach().clone())
    bar = W.detach().clone()
    starts = list(range(0, n_steps, checkpoint_every))
    for seg in reversed(range(len(starts))):
        a = starts[seg]
        b = min(a + checkpoint_every, n_steps)
        Us = ckpt[seg].clone().requires_grad_(True)
        V = Us
        for _ in range(a, b):
            V = dg.rk3_step(V, dt)
        (bar,) = torch.autograd.grad(V, Us, bar)
    return bar
