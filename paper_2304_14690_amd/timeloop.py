"""Time steps of the projection method (Sec. 2.1): the first fractional step
(Eq. 3, pc_momentum_predict), the pressure-correction sub-step with the IB
force warm-started from the previous step (Eqs. 18-20, pc_pressure_correct),
and R^{n-1} for the next step (pc_momentum_pressure).  Buffer management
only: every step runs in the library's kernels."""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import pcorr as pc


class TimeStepper:
    """Advances node velocities [d][M] on one geometry (built with
    k_self > 0) and plan.  mode: PC_F64, PC_F32 or PC_MIXED (the first step
    then runs in float64)."""

    def __init__(self, plan: pc.Plan, geom: pc.Geometry, mode: int, dt: float, nu: float,
                 force: Optional[Sequence[float]] = None, tol: float = 1e-3):
        self.plan, self.geom, self.mode = plan, geom, mode
        self.dt, self.nu, self.force, self.tol = dt, nu, force, tol
        d, M = plan.d, geom.M
        dtype = torch.float32 if mode == pc.PC_F32 else torch.float64
        z = dict(dtype=dtype, device="cuda")
        self.r = torch.zeros((d, M), **z)
        self.r_prev = torch.zeros((d, M), **z)
        self.ustar = torch.zeros((d, M), **z)
        self.p = torch.zeros(plan.G, **z)
        self.g = torch.zeros((d, max(1, geom.n_ib)), **z)
        self.ws = pc.Workspace(plan, geom, mode)
        self.steps = 0
        self.last_stats = None

    def step(self, u: torch.Tensor, u_out: torch.Tensor) -> dict:
        """u -> u_out (they must differ); returns the sub-step statistics."""
        pc.momentum_predict(self.geom, u, self.r_prev if self.steps else None, self.dt,
                            self.nu, self.r, self.ustar, force=self.force)
        g = self.g if self.geom.n_ib else None
        _, st = pc.pressure_correct(self.geom, self.plan, self.mode, self.ustar, self.dt, u_out,
                                    self.p, g=g, tol=self.tol, ws=self.ws)
        pc.momentum_pressure(self.geom, self.r, self.ustar, u_out, g, self.dt, self.r_prev)
        self.steps += 1
        self.last_stats = st
        return st
