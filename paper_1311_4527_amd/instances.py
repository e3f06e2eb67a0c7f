"""Seeded synthetic planning instances.

This module only draws inputs: agent radii, start and goal positions, wall
segments, per-segment cost coefficients and the initial break-point positions.
It holds none of the planner's arithmetic, so the FP64 reference and the GPU
path can both be fed from it.

Workloads follow the paper's numerical section (Sec. 4): CONF1 is the antipodal
circle swap, CONF2 draws starts and goals at random in the plane.  Walls are
static line segments (Sec. 3.2).  Break-point positions are laid out as
``[p][eta+1][dim]``; break-points 0 and eta are the fixed start and goal.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Instance:
    """One planning problem plus the initial break-point positions."""

    p: int
    eta: int
    dim: int
    radii: np.ndarray            # [p]
    x0: np.ndarray               # [p, dim]   start positions x_i(0)
    xT: np.ndarray               # [p, dim]   goal positions x_i(T)
    walls: np.ndarray            # [W, 2, dim] segments (x_L, x_R); dim == 2 only
    C: np.ndarray                # [p, eta] energy coefficient per segment
    z0: np.ndarray               # [p, eta+1, dim] initial break-points
    rho0: float = 1.0
    alpha: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_walls(self) -> int:
        return int(self.walls.shape[0])

    def counts(self) -> dict:
        """Factor / edge / node counts of the factor graph (Sec. 3.3)."""
        p, eta, W = self.p, self.eta, self.n_walls
        fc = eta * p * (p - 1) // 2
        fe = eta * p
        fw = eta * p * W
        ff = 2 * p
        return dict(coll=fc, energy=fe, wall=fw, fixed=ff,
                    factors=fc + fe + fw + ff,
                    edges=4 * fc + 2 * fe + 2 * fw + ff,
                    nodes=(eta + 1) * p)


def _line_init(x0, xT, eta, rng, sigma, dim_noise=None):
    """Straight-line break-points plus N(0, sigma^2) noise on interior ones."""
    p, dim = x0.shape
    s = np.arange(eta + 1, dtype=np.float64) / eta
    z = x0[:, None, :] + s[None, :, None] * (xT - x0)[:, None, :]
    if sigma > 0 and eta > 1:
        noise = rng.normal(0.0, sigma, size=(p, eta - 1, dim))
        if dim_noise is not None:
            noise = noise * dim_noise[None, None, :]
        z[:, 1:eta, :] += noise
    z[:, 0, :] = x0
    z[:, eta, :] = xT
    return z


def circle_swap(p: int, r: float, eta: int, *, dim: int = 2, radius: float = 1.0,
                sigma: float = 1e-3, goal_sigma: float = 0.0, seed: int = 0,
                C: float = 1.0, rho0: float = 1.0, alpha: float = 1.0,
                name: str = "") -> Instance:
    """CONF1: p agents evenly spaced on a circle, each heading to its antipode.

    In 3D the circle lies in the xy-plane and only the init noise leaves it.
    ``goal_sigma`` perturbs the goals (N(0, goal_sigma^2) per coordinate).
    """
    rng = np.random.default_rng(seed)
    ang = 2.0 * np.pi * np.arange(p) / p
    x0 = np.zeros((p, dim))
    x0[:, 0] = radius * np.cos(ang)
    x0[:, 1] = radius * np.sin(ang)
    xT = -x0.copy()
    if goal_sigma > 0:
        xT[:, :2] += rng.normal(0.0, goal_sigma, size=(p, 2))
        # goals must stay pairwise >= 2r apart: redraw the perturbation of
        # the later agent of every overlapping pair until none is left
        for _ in range(10000):
            d2 = np.sum((xT[:, None, :] - xT[None, :, :]) ** 2, axis=2)
            np.fill_diagonal(d2, np.inf)
            bad = np.unique(np.nonzero(np.triu(d2 < (2.0 * r) ** 2))[1])
            if bad.size == 0:
                break
            xT[bad, :2] = -x0[bad, :2] + rng.normal(0.0, goal_sigma, size=(bad.size, 2))
        else:
            raise RuntimeError("goal perturbation did not separate the goals")
    z0 = _line_init(x0, xT, eta, rng, sigma)
    return Instance(p=p, eta=eta, dim=dim, radii=np.full(p, float(r)), x0=x0, xT=xT,
                    walls=np.zeros((0, 2, dim)), C=np.full((p, eta), float(C)), z0=z0,
                    rho0=rho0, alpha=alpha, name=name or f"circle_swap_p{p}_eta{eta}_d{dim}",
                    meta=dict(kind="circle_swap", seed=seed, r=r, sigma=sigma))


def _poisson_points(rng, n, dim, min_sep, lo=0.0, hi=1.0, max_tries=2_000_000):
    pts = np.empty((n, dim))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("rejection sampling did not converge")
        c = rng.uniform(lo, hi, size=dim)
        if k == 0 or np.min(np.sum((pts[:k] - c) ** 2, axis=1)) >= min_sep * min_sep:
            pts[k] = c
            k += 1
    return pts


def _point_segment_dist(P, a, b):
    """Distance from each row of P to segment [a, b] (instance rejection only)."""
    d = b - a
    L2 = float(np.dot(d, d))
    if L2 == 0.0:
        return np.linalg.norm(P - a, axis=1)
    t = np.clip((P - a) @ d / L2, 0.0, 1.0)
    return np.linalg.norm(P - (a + t[:, None] * d), axis=1)


def random_box(p: int, r: float, eta: int, *, n_walls: int = 0, dim: int = 2,
               min_sep: Optional[float] = None, wall_len=(0.05, 0.2), wall_margin: float = 0.002,
               sigma: float = 0.0, seed: int = 0, C: float = 1.0, rho0: float = 1.0,
               alpha: float = 1.0, name: str = "") -> Instance:
    """CONF2-style instance: starts and goals uniform in the unit box.

    Starts (and, separately, goals) are rejection-sampled to pairwise distance
    >= ``min_sep`` (default 2r plus 20%).  Walls: centre uniform in the unit
    square, angle uniform in [0, pi), length uniform in ``wall_len``; a wall
    closer than r + wall_margin to any start or goal is redrawn, so that the
    fixed end points are feasible.
    """
    if n_walls and dim != 2:
        raise ValueError("walls are planar only")
    rng = np.random.default_rng(seed)
    if min_sep is None:
        min_sep = 2.4 * r
    x0 = _poisson_points(rng, p, dim, min_sep)
    xT = _poisson_points(rng, p, dim, min_sep)
    walls = np.zeros((n_walls, 2, dim))
    ends = np.concatenate([x0, xT], axis=0)
    k = 0
    tries = 0
    while k < n_walls:
        tries += 1
        if tries > 100000:
            raise RuntimeError("wall sampling did not converge")
        c = rng.uniform(0.0, 1.0, size=2)
        th = rng.uniform(0.0, np.pi)
        L = rng.uniform(*wall_len)
        h = 0.5 * L * np.array([np.cos(th), np.sin(th)])
        a, b = c - h, c + h
        if np.min(_point_segment_dist(ends, a, b)) < r + wall_margin:
            continue
        walls[k, 0], walls[k, 1] = a, b
        k += 1
    z0 = _line_init(x0, xT, eta, rng, sigma)
    return Instance(p=p, eta=eta, dim=dim, radii=np.full(p, float(r)), x0=x0, xT=xT,
                    walls=walls, C=np.full((p, eta), float(C)), z0=z0, rho0=rho0, alpha=alpha,
                    name=name or f"random_box_p{p}_eta{eta}_W{n_walls}_d{dim}",
                    meta=dict(kind="random_box", seed=seed, r=r, min_sep=min_sep))


# ---------------------------------------------------------------------------
# The five workloads used throughout the tests and the benchmark.
#
# Step size alpha = 0.1 and the energy prefactor 1/(p eta) follow the paper
# (Sec. 4 and eq. velo_cost_pair_wise); rho0 = 1.
# ---------------------------------------------------------------------------

PAPER_ALPHA = 0.1


def _paper_C(p, eta):
    return 1.0 / (p * eta)

def conf_small(seed: int = 0) -> Instance:
    """p=8 circle swap, r=0.05, eta=4, init noise sigma=1e-3."""
    return circle_swap(8, 0.05, 4, sigma=1e-3, seed=seed, alpha=PAPER_ALPHA, C=_paper_C(8, 4),
                       name=f"swap8_eta4_s{seed}")


def conf_swap100(seed: int = 0) -> Instance:
    """p=100 circle swap, r=0.02, eta=8 (39,600 collision factors)."""
    return circle_swap(100, 0.02, 8, sigma=1e-3, seed=seed, alpha=PAPER_ALPHA, C=_paper_C(100, 8),
                       name=f"swap100_eta8_s{seed}")


def conf_box1024(seed: int = 1234, p: int = 1024, eta: int = 16, n_walls: int = 32) -> Instance:
    """p=1024 random box, r=0.005, >=0.012 separation, 32 walls, eta=16."""
    return random_box(p, 0.005, eta, n_walls=n_walls, min_sep=0.012, sigma=0.0, seed=seed,
                      alpha=PAPER_ALPHA, C=_paper_C(p, eta), name=f"box{p}_eta{eta}_W{n_walls}_s{seed}")


def conf_batch(n: int = 256, base_seed: int = 2024, p_range=(4, 128)) -> List[Instance]:
    """Ragged batch: p ~ U{4..128}, eta in {4,8,16}; half circle swaps, half
    random boxes (0-8 walls, planar only), r=0.01; half of each kind in 3D."""
    out = []
    for b in range(n):
        rng = np.random.default_rng(base_seed + b)
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        eta = int(rng.choice([4, 8, 16]))
        dim = 3 if (b // 2) % 2 == 1 else 2
        if b % 2 == 0:
            if p % 2:
                p += 1
            inst = circle_swap(p, 0.01, eta, dim=dim, sigma=1e-3, seed=base_seed + b, alpha=PAPER_ALPHA,
                               C=_paper_C(p, eta), name=f"batch{b}_swap{p}_eta{eta}_d{dim}")
        else:
            nw = int(rng.integers(0, 9)) if dim == 2 else 0
            inst = random_box(p, 0.01, eta, n_walls=nw, dim=dim, min_sep=0.024, sigma=1e-3,
                              seed=base_seed + b, alpha=PAPER_ALPHA, C=_paper_C(p, eta),
                              name=f"batch{b}_box{p}_eta{eta}_W{nw}_d{dim}")
        out.append(inst)
    return out


def conf_adjoint(seed: int = 7, p: int = 256) -> Instance:
    """p=256 circle swap, r=0.008, eta=8, goals perturbed by N(0, 0.01^2)."""
    return circle_swap(p, 0.008, 8, sigma=1e-3, goal_sigma=0.01, seed=seed, alpha=PAPER_ALPHA,
                       C=_paper_C(p, 8), name=f"swap{p}_eta8_goalnoise_s{seed}")


def sub_instance(inst: Instance, agents) -> Instance:
    """Restrict an instance to a subset of agents (same eta, walls, init)."""
    agents = np.asarray(agents)
    return Instance(p=len(agents), eta=inst.eta, dim=inst.dim, radii=inst.radii[agents].copy(),
                    x0=inst.x0[agents].copy(), xT=inst.xT[agents].copy(), walls=inst.walls.copy(),
                    C=inst.C[agents].copy(), z0=inst.z0[agents].copy(), rho0=inst.rho0,
                    alpha=inst.alpha, name=inst.name + f"_sub{len(agents)}", meta=dict(inst.meta))


def random_state(inst: Instance, seed: int, u_scale: float = 1e-2, active_frac: float = 0.5):
    """A random (z, u, ←rho) state for single-iteration checks.

    z: the instance's init plus N(0, (u_scale)^2) on interior break-points;
    u: N(0, u_scale^2) per edge coordinate, zeroed on a random ``1-active_frac``
    of the factors and on every edge touching an end point (their u is zero in
    any reachable state).  Returns u in the canonical edge order described in
    the public header.  ←rho is the default (INF at end points, STD inside).
    """
    rng = np.random.default_rng(seed)
    c = inst.counts()
    p, eta, d = inst.p, inst.eta, inst.dim
    z = inst.z0.copy()
    if eta > 1:
        z[:, 1:eta] += rng.normal(0.0, u_scale, size=(p, eta - 1, d))
    u = rng.normal(0.0, u_scale, size=(c["edges"], d))
    # edge -> (agent, break-point) in canonical order, to zero end-point edges
    nodes = canonical_edge_nodes(inst)
    s_of_edge = nodes % (eta + 1)
    u[(s_of_edge == 0) | (s_of_edge == eta)] = 0.0
    # zero whole factors at random (inactive ones carry u = 0)
    fac = canonical_edge_factor(inst)
    keep = rng.uniform(size=c["factors"]) < active_frac
    u[~keep[fac]] = 0.0
    lrho = np.full((p, eta + 1), 1, dtype=np.uint8)
    lrho[:, 0] = 2
    lrho[:, eta] = 2
    return z, u, lrho


def canonical_edge_nodes(inst: Instance) -> np.ndarray:
    """Node id (agent*(eta+1) + s) of every edge, in the canonical edge order:
    fixed (start i, goal i) for each i; energy (i, s); collision (s, i<j) with
    edges [(i,s),(i,s+1),(j,s),(j,s+1)]; wall (s, i, w) with [(i,s),(i,s+1)]."""
    p, eta, W = inst.p, inst.eta, inst.n_walls
    E1 = eta + 1
    out = []
    i = np.arange(p)
    fx = np.stack([i * E1, i * E1 + eta], axis=1).reshape(-1)
    out.append(fx)
    ii, ss = np.meshgrid(np.arange(p), np.arange(eta), indexing="ij")
    en = np.stack([ii * E1 + ss, ii * E1 + ss + 1], axis=-1).reshape(-1)
    out.append(en)
    iu, ju = np.triu_indices(p, 1)
    for s in range(eta):
        cn = np.stack([iu * E1 + s, iu * E1 + s + 1, ju * E1 + s, ju * E1 + s + 1], axis=1)
        out.append(cn.reshape(-1))
    if W:
        for s in range(eta):
            a = np.repeat(np.arange(p), W)
            wn = np.stack([a * E1 + s, a * E1 + s + 1], axis=1)
            out.append(wn.reshape(-1))
    return np.concatenate(out).astype(np.int64)


def canonical_edge_factor(inst: Instance) -> np.ndarray:
    """Factor id of every edge in canonical order (factors ordered as the edges)."""
    c = inst.counts()
    per = np.concatenate([np.full(c["fixed"], 1), np.full(c["energy"], 2),
                          np.full(c["coll"], 4), np.full(c["wall"], 2)])
    return np.repeat(np.arange(c["factors"]), per)
