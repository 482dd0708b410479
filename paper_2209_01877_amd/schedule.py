"""Temporal mixed precision (the paper's MP-N scheme, Sec. III.B, Table 2): the first
n_low SSP-RK3 steps run in a low-precision mode, the remaining steps in FP64.

The two discretisations share the mesh; the state passes between them through the
caller-order layout (tdg_get_state / tdg_set_state), so each may use its own internal
numbering.  All arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import torch

from .solver import Solver


class TemporalMixed:
    def __init__(self, p: int, mesh, low: str = "fp32", high: str = "fp64", renumber: str = "hilbert",
                 farfield=None, flux: str = "rusanov"):
        self.low = Solver(p, low)
        self.high = Solver(p, high)
        for s in (self.low, self.high):
            s.upload(mesh, renumber=renumber)
            if farfield is not None:
                s.set_farfield(farfield)
            s.set_flux(flux)
        self.work_low = self.low.new_work()
        self.work_high = self.high.new_work()

    def run(self, U_user: torch.Tensor, dt: float, n_low: int, n_total: int) -> torch.Tensor:
        """Advance a caller-layout FP64 state by n_total steps, the first n_low in low precision."""
        assert 0 <= n_low <= n_total
        U = U_user
        if n_low > 0:
            Ul = self.low.set_state(U_user.contiguous())
            self.low.rk_step(Ul, dt, n_low, self.work_low)
            U = self.low.get_state(Ul)
        if n_total > n_low:
            Uh = self.high.set_state(U.contiguous())
            self.high.rk_step(Uh, dt, n_total - n_low, self.work_high)
            U = self.high.get_state(Uh)
        return U
