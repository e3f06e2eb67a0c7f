"""Brute-force checkers for the minimisers (test-only, independent of the
reference and of the GPU path).

Each solves the minimiser's defining problem directly: a weighted squared
distance to the incoming n-messages subject to the non-collision constraint,
by multi-start SLSQP, or scans a 1-D formulation densely.
"""
import numpy as np
from scipy.optimize import minimize


def cpa_np(d0, d1):
    """Closest approach of (1-a) d0 + a d1 over a in [0,1] (closed form)."""
    d0 = np.asarray(d0, float)
    e = np.asarray(d1, float) - d0
    ee = float(e @ e)
    a = 0.0 if ee == 0 else float(np.clip(-(d0 @ e) / ee, 0.0, 1.0))
    return float(np.linalg.norm(d0 + a * e))


def cpa_sampled(d0, d1, n=200001):
    a = np.linspace(0.0, 1.0, n)[:, None]
    return float(np.min(np.linalg.norm((1 - a) * np.asarray(d0) + a * np.asarray(d1), axis=1)))


def segseg_sampled(p0, p1, q0, q1, n=2001):
    a = np.linspace(0.0, 1.0, n)
    P = (1 - a)[:, None] * np.asarray(p0) + a[:, None] * np.asarray(p1)
    Q = (1 - a)[:, None] * np.asarray(q0) + a[:, None] * np.asarray(q1)
    best = np.inf
    for k in range(0, n, 200):
        blk = P[k:k + 200]
        d = np.linalg.norm(blk[:, None, :] - Q[None, :, :], axis=2)
        best = min(best, float(d.min()))
    return best


def point_seg(q, a, b):
    q, a, b = (np.asarray(v, float) for v in (q, a, b))
    d = b - a
    L2 = d @ d
    t = 0.0 if L2 == 0 else float(np.clip((q - a) @ d / L2, 0, 1))
    return float(np.linalg.norm(a + t * d - q))


def segseg_closed(p0, p1, q0, q1):
    """Planar segment distance: 0 if they cross, else the least of the four
    end-point-to-segment distances."""
    p0, p1, q0, q1 = (np.asarray(v, float) for v in (p0, p1, q0, q1))

    def cross(a, b):
        return a[0] * b[1] - a[1] * b[0]
    r, s = p1 - p0, q1 - q0
    den = cross(r, s)
    if den != 0:
        t = cross(q0 - p0, s) / den
        u = cross(q0 - p0, r) / den
        if 0 <= t <= 1 and 0 <= u <= 1:
            return 0.0
    return min(point_seg(p0, q0, q1), point_seg(p1, q0, q1), point_seg(q0, p0, p1), point_seg(q1, p0, p1))


def segseg_exact(p0, p1, q0, q1):
    """Planar segment distance via minimisation over the 2-D parameter box."""
    p0, p1, q0, q1 = (np.asarray(v, float) for v in (p0, p1, q0, q1))
    # distance is a convex function of (a, b): project-and-minimise
    def f(ab):
        a, b = np.clip(ab, 0, 1)
        return np.sum(((1 - a) * p0 + a * p1 - (1 - b) * q0 - b * q1) ** 2)
    best = np.inf
    for s in ([0.5, 0.5], [0, 0], [1, 1], [0, 1], [1, 0]):
        r = minimize(f, s, method="L-BFGS-B", bounds=[(0, 1), (0, 1)], options=dict(ftol=1e-16, gtol=1e-14))
        best = min(best, r.fun)
    return float(np.sqrt(max(best, 0.0)))


def brute_coll(n, w, R, rng, starts=40):
    """min sum_k (w_k/2)|x_k - n_k|^2 s.t. closest approach of agent 2 minus
    agent 1 over the segment >= R.  n rows: (n_lo, n_hi, n_lo', n_hi').
    Returns (energy, x) of the best feasible local optimum found."""
    n = np.asarray(n, float)
    d = n.shape[1]
    w = np.asarray(w, float)

    def f(x):
        x = x.reshape(4, d)
        return 0.5 * float(np.sum(w[:, None] * (x - n) ** 2))

    def jac(x):
        x = x.reshape(4, d)
        return (w[:, None] * (x - n)).reshape(-1)

    def g(x):
        x = x.reshape(4, d)
        return cpa_np(x[2] - x[0], x[3] - x[1]) - R

    best = None
    for t in range(starts):
        x0 = n.reshape(-1) + rng.normal(0, R * (0.3 + t / starts), n.size)
        res = minimize(f, x0, jac=jac, constraints=[{"type": "ineq", "fun": g}], method="SLSQP",
                       options=dict(maxiter=500, ftol=1e-15))
        x = res.x.reshape(4, d)
        if g(res.x) < -1e-9:
            continue
        if best is None or res.fun < best[0]:
            best = (res.fun, x)
    return best


def brute_capsule(xL, xR, r, n, w, rng, starts=40):
    """min sum_k (w_k/2)|x_k - n_k|^2 s.t. dist([x0,x1],[xL,xR]) >= r."""
    n = np.asarray(n, float)
    w = np.asarray(w, float)

    def f(x):
        x = x.reshape(2, 2)
        return 0.5 * float(np.sum(w[:, None] * (x - n) ** 2))

    def jac(x):
        x = x.reshape(2, 2)
        return (w[:, None] * (x - n)).reshape(-1)

    def g(x):
        x = x.reshape(2, 2)
        return segseg_closed(x[0], x[1], xL, xR) - r

    best = None
    for t in range(starts):
        x0 = n.reshape(-1) + rng.normal(0, r * (0.3 + 2 * t / starts), 4)
        res = minimize(f, x0, jac=jac, constraints=[{"type": "ineq", "fun": g}], method="SLSQP",
                       options=dict(maxiter=400, ftol=1e-15))
        if g(res.x) < -1e-9:
            continue
        if best is None or res.fun < best[0]:
            best = (res.fun, res.x.reshape(2, 2))
    return best


def separating_scan(xL, xR, r, n, w, N=200000):
    """Independent 1-D characterisation of the capsule minimiser.

    A segment avoids the open capsule iff some line separates them, i.e. iff
    both ends lie in {x: <x, u> >= h(u)} for a unit u, h the capsule's
    support function.  For fixed u the best ends are the projections of n
    onto that half-plane, so the optimum energy is
        min_u sum_k (w_k/2) max(0, h(u) - <n_k, u>)^2.
    Scanned on N angles, then refined by golden-section on the best cell."""
    xL = np.asarray(xL, float)
    xR = np.asarray(xR, float)
    n = np.asarray(n, float)
    w = np.asarray(w, float)

    def F(th):
        th = np.atleast_1d(th)
        u = np.stack([np.cos(th), np.sin(th)], axis=-1)
        h = np.maximum(u @ xL, u @ xR) + r
        gap = np.maximum(0.0, h[:, None] - u @ n.T)
        return 0.5 * (gap ** 2 @ w)

    th = np.linspace(0, 2 * np.pi, N, endpoint=False)
    vals = F(th)
    k = int(np.argmin(vals))
    a, b = th[k] - 2 * np.pi / N, th[k] + 2 * np.pi / N
    g = (np.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = b - g * (b - a), a + g * (b - a)
        if F(c)[0] < F(d)[0]:
            b = d
        else:
            a = c
    return float(min(F(0.5 * (a + b))[0], vals[k]))


def brute_vel(nl, nh, wl, wh, C, minimum, starts=12, seed=0):
    """min (wl/2)|xl-nl|^2 + (wh/2)|xh-nh|^2 s.t. |xl-xh| <= C (or >= C for
    the minimum-velocity constraint), multi-start SLSQP."""
    nl, nh = np.asarray(nl, float), np.asarray(nh, float)
    dim = nl.shape[0]
    rng = np.random.default_rng(seed)

    def f(v):
        return 0.5 * wl * np.sum((v[:dim] - nl) ** 2) + 0.5 * wh * np.sum((v[dim:] - nh) ** 2)

    def g(v):
        dd = np.sum((v[:dim] - v[dim:]) ** 2)
        return (dd - C * C) if minimum else (C * C - dd)

    best = None
    for k in range(starts):
        x0 = np.concatenate([nl, nh]) + rng.normal(0, 0.3 * (C + 1e-3), 2 * dim) * (k > 0)
        r = minimize(f, x0, constraints=[dict(type="ineq", fun=g)], method="SLSQP",
                     options=dict(ftol=1e-14, maxiter=500))
        if g(r.x) < -1e-9:
            continue
        if best is None or r.fun < best.fun:
            best = r
    return best.x[:dim], best.x[dim:], best.fun


def brute_vo_epoch(x0, xref, radii, c, starts=60, seed=0):
    """Velocity-obstacle epoch (eq. rec_col_avoi_pos): min sum_i c_i |x_i - xref_i|^2
    s.t. every pair moving at constant velocity from x0 to x stays >= r_i + r_j
    apart, by multi-start SLSQP on the exact closest-approach constraint."""
    x0, xref = np.asarray(x0, float), np.asarray(xref, float)
    p, dim = x0.shape
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(p, 1)

    def f(v):
        return float(np.sum(c[:, None] * (v.reshape(p, dim) - xref) ** 2))

    def g(v):
        x = v.reshape(p, dim)
        out = []
        for i, j in zip(iu, ju):
            out.append(cpa_np(x0[j] - x0[i], x[j] - x[i]) - (radii[i] + radii[j]))
        return np.array(out)

    best = None
    for k in range(starts):
        v0 = (xref + rng.normal(0, 0.3 * float(np.max(radii)) * (k > 0) * 4, xref.shape)).reshape(-1)
        r = minimize(f, v0, constraints=[dict(type="ineq", fun=g)], method="SLSQP",
                     options=dict(ftol=1e-13, maxiter=1000))
        if np.min(g(r.x)) < -1e-8:
            continue
        if best is None or r.fun < best.fun:
            best = r
    return best.x.reshape(p, dim), best.fun
