"""Differentiable planner: ``TWASolve`` runs K iterations of the planner on
the GPU and differentiates them with the library's adjoint (twa_backward),
so a loss of the final trajectories can be back-propagated to the starts,
goals, radii and the initial break-points.

The derivative holds every discrete decision of the forward run fixed (the
0 / rho0 / infinity weights and the candidate each minimiser took), as the
unrolled map is piecewise smooth in its inputs.  Planar (dim 2) only.
"""
from __future__ import annotations

from typing import Optional

import torch

from .twa import Solver, TWA_F_TAPE


class TWASolve(torch.autograd.Function):
    """z^K = TWASolve.apply(x0, xT, radii, z0, K, C, walls, rho0, alpha)

    x0, xT [p][2], radii [p], z0 [p][eta+1][2] (break-points 0 and eta are
    replaced by x0 and xT), C [p][eta], walls [W][2][2] or None."""

    @staticmethod
    def forward(ctx, x0, xT, radii, z0, K: int, C, walls, rho0: float, alpha: float):
        p, eta1, dim = z0.shape
        S = Solver(p, eta1 - 1, dim, radii.detach(), x0.detach(), xT.detach(),
                   walls=None if walls is None else walls.detach(), C=C.detach(), rho0=rho0, alpha=alpha,
                   flags=TWA_F_TAPE, device=z0.device)
        S.twa_set_init(z0.detach())
        S.twa_iterate(int(K))
        z = S.twa_get_trajectories()
        ctx.solver = S
        return z

    @staticmethod
    def backward(ctx, gz):
        S = ctx.solver
        dx0, dxT, dr, dz0 = S.twa_backward(gz.contiguous(), want_dz0=True)
        S.close()
        ctx.solver = None
        return dx0, dxT, dr, dz0, None, None, None, None, None


def straight_line(x0: torch.Tensor, xT: torch.Tensor, eta: int) -> torch.Tensor:
    """Break-points evenly spaced on the segment from x0 to xT: [p][eta+1][dim]."""
    t = torch.linspace(0.0, 1.0, eta + 1, device=x0.device, dtype=x0.dtype).view(1, -1, 1)
    return x0.unsqueeze(1) + t * (xT - x0).unsqueeze(1)


def solve(x0: torch.Tensor, xT: torch.Tensor, radii: torch.Tensor, K: int, eta: int,
          C: Optional[torch.Tensor] = None, walls: Optional[torch.Tensor] = None,
          z0: Optional[torch.Tensor] = None, rho0: float = 1.0, alpha: float = 0.1) -> torch.Tensor:
    """Differentiable z^K; z0 defaults to straight lines (itself a function of
    x0 and xT, so their gradients include that path)."""
    if z0 is None:
        z0 = straight_line(x0, xT, eta)
    if C is None:
        C = torch.ones((x0.shape[0], eta), device=x0.device)
    return TWASolve.apply(x0, xT, radii, z0, int(K), C, walls, float(rho0), float(alpha))
