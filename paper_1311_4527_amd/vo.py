"""Velocity-obstacle local planner (Sec. 5): every epoch solves, on the GPU,
the joint problem of eq. rec_col_avoi_pos for new end positions x_i after a
horizon tau, closest to the preferred ones x^ref_i = x_i(0) + v^ref_i tau
without any two agents colliding while moving there at constant velocity
(and without touching a wall); the agents then move a fraction of the way
and the next epoch starts from there.  One solver created with TWA_F_VO
(eta = 1) serves every epoch: each epoch loads its start and reference end
positions (twa_set_endpoints) and iterates until the device's clearance
measure says the plan is collision-free (twa_iterate_until: for a small
instance the whole epoch, checks included, is one persistent launch); this
module only drives the epochs.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .twa import Solver, TWAError, TWA_E_INVALID, TWA_F_VO


class VOPlanner:
    """Epoch loop of the velocity-obstacle planner.

    positions, goals [p][dim]; radii [p]; walls [W][2][2] or None.
    tau: horizon of an epoch; fraction: share of the epoch executed before
    replanning (the paper's alpha of Sec. 5); vmax: preferred speed;
    cost: c_i per agent (default 0.01 (1 + 0.001 i): slightly different
    costs break the symmetry of antipodal swaps, Sec. 5, and a deviation
    cost well below rho0 lets crowded epochs converge); iters: cap on the
    planner iterations of one epoch, which runs in blocks of `check`
    iterations until its plan is collision-free (the paper times each epoch
    to convergence; the check runs on the device); margin: relative safety
    margin on the radii used for
    planning, so that a plan that is collision-free up to FP32 rounding
    keeps the agents strictly apart at their true radii."""

    def __init__(self, positions, goals, radii, walls=None, tau: float = 1.0, fraction: float = 0.5,
                 vmax: float = 0.25, cost=None, rho0: float = 1.0, alpha: float = 0.1, iters: int = 20000,
                 check: int = 50, margin: float = 1e-3, device="cuda"):
        self.pos = np.asarray(positions, dtype=np.float64).copy()
        self.goals = np.asarray(goals, dtype=np.float64).copy()
        self.radii = np.asarray(radii, dtype=np.float64)
        self.p, self.dim = self.pos.shape
        self.walls = None if walls is None else np.asarray(walls, dtype=np.float64)
        self.tau, self.fraction, self.vmax = float(tau), float(fraction), float(vmax)
        self.cost = (0.01 * (1.0 + 0.001 * np.arange(self.p))) if cost is None else np.asarray(cost, float)
        self.rho0, self.alpha, self.device = rho0, alpha, device
        self.iters, self.check = int(iters), max(1, int(check))
        self.plan_radii = self.radii * (1.0 + float(margin))
        self.last_iterations = 0     # iterations the last epoch took (0: cap reached)
        self._S = None               # the epochs' solver

    def reference(self) -> np.ndarray:
        """x^ref: straight towards the goal at up to vmax for tau."""
        d = self.goals - self.pos
        dist = np.linalg.norm(d, axis=1)
        speed = np.minimum(dist / self.tau, self.vmax)
        v = d / np.maximum(dist, 1e-12)[:, None] * speed[:, None]
        return self.pos + v * self.tau

    def clearance(self, a: np.ndarray, b: np.ndarray, radii: Optional[np.ndarray] = None) -> float:
        """Smallest closest approach minus (r_i + r_j) when every agent moves
        at constant velocity from a to b (positive: collision-free), and the
        smallest distance minus r_i from any wall along the way (2-D)."""
        R = self.radii if radii is None else radii
        out = np.inf
        if self.p > 1:
            iu, ju = np.triu_indices(self.p, 1)
            d0 = a[ju] - a[iu]
            e = (b[ju] - b[iu]) - d0
            ee = np.sum(e * e, axis=1)
            t = np.clip(-np.sum(d0 * e, axis=1) / np.where(ee > 0, ee, 1.0), 0.0, 1.0)
            v = d0 + t[:, None] * e
            out = float(np.min(np.sqrt(np.sum(v * v, axis=1)) - (R[iu] + R[ju])))
        if self.walls is not None and len(self.walls):
            for w in self.walls:
                for i in range(self.p):
                    out = min(out, _seg_seg_distance(a[i], b[i], w[0], w[1]) - R[i])
        return out

    def _plan_ok(self, x: np.ndarray) -> bool:
        # collision-free at the planning radii up to FP32 rounding of the
        # positions (relative 5e-6, inside what the solver accepts as starts)
        return self.clearance(self.pos, x, self.plan_radii * (1.0 - 5e-6)) >= 0.0

    def _solver(self, xref: np.ndarray) -> Solver:
        """The epochs' solver with this epoch's start and reference ends
        (made at the first epoch, and again should an agent leave the
        coordinate range it was made for)."""
        if self._S is not None:
            try:
                self._S.twa_set_endpoints(self.pos, xref)
                return self._S
            except TWAError as e:
                if e.status != TWA_E_INVALID:
                    raise
                self._S.close()
        self._S = Solver(self.p, 1, self.dim, self.plan_radii, self.pos, xref, walls=self.walls,
                         C=self.cost[:, None], rho0=self.rho0, alpha=self.alpha, flags=TWA_F_VO, device=self.device)
        return self._S

    def solve_epoch(self, xref: Optional[np.ndarray] = None) -> np.ndarray:
        """End positions of one epoch (break-point 1 of the solver), iterated
        until collision-free or the iteration cap."""
        xref = self.reference() if xref is None else xref
        S = self._solver(xref)
        # collision-free at the planning radii up to FP32 rounding of the
        # positions (relative 5e-6, inside what the solver accepts as starts)
        tol = -1e-5 * float(self.plan_radii.min())
        done, met = S.twa_iterate_until(self.iters, self.check, tol)
        self.last_iterations = done if met else 0
        return S.twa_get_trajectories()[:, 1].cpu().numpy().astype(np.float64)

    def close(self):
        if self._S is not None:
            self._S.close()
            self._S = None

    def step(self) -> np.ndarray:
        """Plan one epoch and move a fraction of the way; returns the new
        positions.  Should the epoch stop at its cap short of a collision-free
        plan, the executed share is halved until the motion is collision-free
        (staying put always is)."""
        x = self.solve_epoch()
        t = self.fraction
        new = self.pos.copy()
        for _ in range(30):
            cand = self.pos + t * (x - self.pos)
            if self._plan_ok(cand):
                new = cand
                break
            t *= 0.5
        self.pos = new
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


def _seg_seg_distance(a0, a1, b0, b1) -> float:
    """Distance between the 2-D segments [a0, a1] and [b0, b1]."""
    def pt_seg(q, s0, s1):
        d = s1 - s0
        L2 = float(d @ d)
        t = 0.0 if L2 <= 0 else min(1.0, max(0.0, float((q - s0) @ d) / L2))
        return float(np.linalg.norm(s0 + t * d - q))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    d1, d2 = cross(b0, b1, a0), cross(b0, b1, a1)
    d3, d4 = cross(a0, a1, b0), cross(a0, a1, b1)
    if ((d1 > 0) != (d2 > 0)) and ((d3 > 0) != (d4 > 0)) and d1 != 0 and d2 != 0 and d3 != 0 and d4 != 0:
        return 0.0
    return min(pt_seg(a0, b0, b1), pt_seg(a1, b0, b1), pt_seg(b0, a0, a1), pt_seg(b1, a0, a1))
