"""Velocity-obstacle local planner (Sec. 5): every epoch solves, on the GPU,
the joint problem of eq. rec_col_avoi_pos for new end positions x_i after a
horizon tau, closest to the preferred ones x^ref_i = x_i(0) + v^ref_i tau
without any two agents colliding while moving there at constant velocity
(and without touching a wall); the agents then move a fraction of the way
and the next epoch starts from there.  Each epoch is one solver created with
TWA_F_VO (eta = 1); this module only drives the epochs.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .twa import Solver, TWA_F_VO


class VOPlanner:
    """Epoch loop of the velocity-obstacle planner.

    positions, goals [p][dim]; radii [p]; walls [W][2][2] or None.
    tau: horizon of an epoch; fraction: share of the epoch executed before
    replanning (the paper's alpha of Sec. 5); vmax: preferred speed;
    cost: c_i per agent (default 0.1 (1 + 0.001 i): slightly different
    costs break the symmetry of antipodal swaps, Sec. 5); iters: planner
    iterations per epoch."""

    def __init__(self, positions, goals, radii, walls=None, tau: float = 1.0, fraction: float = 0.5,
                 vmax: float = 0.25, cost=None, rho0: float = 1.0, alpha: float = 0.1, iters: int = 1500,
                 device="cuda"):
        self.pos = np.asarray(positions, dtype=np.float64).copy()
        self.goals = np.asarray(goals, dtype=np.float64).copy()
        self.radii = np.asarray(radii, dtype=np.float64)
        self.p, self.dim = self.pos.shape
        self.walls = None if walls is None else np.asarray(walls, dtype=np.float64)
        self.tau, self.fraction, self.vmax = float(tau), float(fraction), float(vmax)
        self.cost = (0.1 * (1.0 + 0.001 * np.arange(self.p))) if cost is None else np.asarray(cost, float)
        self.rho0, self.alpha, self.iters, self.device = rho0, alpha, int(iters), device

    def reference(self) -> np.ndarray:
        """x^ref: straight towards the goal at up to vmax for tau."""
        d = self.goals - self.pos
        dist = np.linalg.norm(d, axis=1)
        speed = np.minimum(dist / self.tau, self.vmax)
        v = d / np.maximum(dist, 1e-12)[:, None] * speed[:, None]
        return self.pos + v * self.tau

    def solve_epoch(self, xref: Optional[np.ndarray] = None) -> np.ndarray:
        """End positions of one epoch (break-point 1 of the solver)."""
        xref = self.reference() if xref is None else xref
        S = Solver(self.p, 1, self.dim, self.radii, self.pos, xref, walls=self.walls, C=self.cost[:, None],
                   rho0=self.rho0, alpha=self.alpha, flags=TWA_F_VO, device=self.device)
        S.twa_set_init(np.stack([self.pos, xref], axis=1))
        S.twa_iterate(self.iters)
        x = S.twa_get_trajectories()[:, 1].cpu().numpy().astype(np.float64)
        S.close()
        return x

    def step(self) -> np.ndarray:
        """Plan one epoch and move a fraction of the way; returns the new positions."""
        x = self.solve_epoch()
        self.pos = self.pos + self.fraction * (x - self.pos)
        return self.pos

    def arrived(self, tol: float = 1e-2) -> bool:
        return bool(np.all(np.linalg.norm(self.goals - self.pos, axis=1) < tol))

    def run(self, max_epochs: int = 200, tol: float = 1e-2):
        """Epochs until every agent is within tol of its goal; returns the
        positions after every epoch (including the start)."""
        path = [self.pos.copy()]
        for _ in range(max_epochs):
            if self.arrived(tol):
                break
            path.append(self.step().copy())
        torch.cuda.synchronize()
        return path
