"""ctypes wrapper of the FP64 reference planner (``libtwa_oracle.so``).

TEST INFRASTRUCTURE ONLY.  Every function mirrors one C entry point of
``twa_oracle.c``; see that file for the steps (App. B of the paper) and the
minimisers (App. C-E, App. I) each one follows.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtwa_oracle.so")

ZERO, STD, INF = 0, 1, 2
MODE_TWA, MODE_ADMM = 0, 1
COST_ENERGY, COST_NONE, COST_MAXVEL, COST_MINVEL, COST_VO = 0, 1, 2, 3, 4

_lib = None
_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int)
_u8 = ct.POINTER(ct.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .build import build
        build()
    lib = ct.CDLL(LIB_PATH)
    lib.tor_cpa.restype = ct.c_double
    lib.tor_cpa.argtypes = [_dp, _dp, ct.c_int]
    lib.tor_segseg.restype = ct.c_double
    lib.tor_segseg.argtypes = [_dp, _dp, _dp, _dp]
    lib.tor_prox_energy.restype = None
    lib.tor_prox_energy.argtypes = [_dp, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int, _dp, _dp]
    lib.tor_prox_vel.restype = ct.c_int
    lib.tor_prox_vel.argtypes = [_dp, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_int, ct.c_int, _dp, _dp]
    lib.tor_prox_capsule.restype = ct.c_int
    lib.tor_prox_capsule.argtypes = [_dp, _dp, ct.c_double, _dp, _dp, ct.c_double, ct.c_double, _dp, _dp,
                                     _ip, _dp]
    lib.tor_prox_coll.restype = ct.c_int
    lib.tor_prox_coll.argtypes = [_dp, _dp, _dp, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                  ct.c_double, ct.c_int, _dp, _dp, _dp, _dp, _ip, _dp]
    lib.tor_create.restype = ct.c_void_p
    lib.tor_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, _dp, _dp, _dp, ct.c_int, _dp, _dp,
                               ct.c_double, ct.c_double, ct.c_int, ct.c_int]
    lib.tor_destroy.restype = None
    lib.tor_destroy.argtypes = [ct.c_void_p]
    for nm in ("tor_num_factors", "tor_num_edges", "tor_iteration"):
        getattr(lib, nm).restype = ct.c_long
        getattr(lib, nm).argtypes = [ct.c_void_p]
    lib.tor_set_schedule.restype = None
    lib.tor_set_schedule.argtypes = [ct.c_void_p, ct.c_double, ct.c_int]
    lib.tor_set_state.restype = None
    lib.tor_set_state.argtypes = [ct.c_void_p, _dp, _dp, _u8, ct.c_long]
    lib.tor_get_state.restype = None
    lib.tor_get_state.argtypes = [ct.c_void_p, _dp, _dp, _u8]
    lib.tor_get_last.restype = None
    lib.tor_get_last.argtypes = [ct.c_void_p, _dp, _u8]
    lib.tor_iterate.restype = None
    lib.tor_iterate.argtypes = [ct.c_void_p, ct.c_long]
    lib.tor_get_margins.restype = None
    lib.tor_get_margins.argtypes = [ct.c_void_p, _dp, _dp]
    lib.tor_override_next.restype = None
    lib.tor_override_next.argtypes = [ct.c_void_p, ct.c_long, ct.POINTER(ct.c_long), _dp, _u8]
    lib.tor_prox_capsule_gap.restype = ct.c_int
    lib.tor_prox_capsule_gap.argtypes = [_dp, _dp, ct.c_double, _dp, _dp, ct.c_double, ct.c_double, _dp, _dp,
                                         _ip, _dp, _dp]
    lib.tor_prox_coll_gap.restype = ct.c_int
    lib.tor_prox_coll_gap.argtypes = [_dp, _dp, _dp, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                      ct.c_double, ct.c_int, _dp, _dp, _dp, _dp, _ip, _dp, _dp]
    lib.tor_tape.restype = ct.c_long
    lib.tor_tape.argtypes = [ct.c_void_p, ct.c_long]
    lib.tor_backward.restype = None
    lib.tor_backward.argtypes = [ct.c_void_p, _dp, _dp, _dp, _dp, _dp]
    lib.tor_objective.restype = ct.c_double
    lib.tor_objective.argtypes = [ct.c_void_p]
    lib.tor_min_clearance.restype = ct.c_double
    lib.tor_min_clearance.argtypes = [ct.c_int, ct.c_int, ct.c_int, _dp, _dp, ct.c_int, _dp]
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    """Threads of the reference's OpenMP loops (the runtime it links)."""
    _load()
    ct.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _w(x):
    """weight argument: a float, or ``np.inf`` for the certain weight"""
    return float(x)


# ------------------------------------------------------------------ geometry

def cpa(d0, d1) -> float:
    """min over alpha in [0,1] of |(1-alpha) d0 + alpha d1| (eq. basic_opt_prob)."""
    a, pa = _d(d0)
    b, pb = _d(d1)
    return _load().tor_cpa(pa, pb, a.shape[0])


def segseg(p0, p1, q0, q1) -> float:
    """distance between planar segments (the constraint of eq. wall_minimizer)."""
    arrs = [_d(v) for v in (p0, p1, q0, q1)]
    return _load().tor_segseg(*[x[1] for x in arrs])


# ---------------------------------------------------------------- minimisers

def prox_energy(nl, nh, wl, wh, C):
    """Energy minimiser, App. E: returns (x_lo, x_hi)."""
    a, pa = _d(nl)
    b, pb = _d(nh)
    xl = np.zeros_like(a)
    xh = np.zeros_like(a)
    _load().tor_prox_energy(pa, pb, _w(wl), _w(wh), float(C), a.shape[0], xl.ctypes.data_as(_dp),
                            xh.ctypes.data_as(_dp))
    return xl, xh


def prox_vel(nl, nh, wl, wh, C, minimum: bool):
    """Maximum (minimum) velocity minimiser, App. F (App. G): returns
    (binding, x_lo, x_hi)."""
    a, pa = _d(nl)
    b, pb = _d(nh)
    xl = np.zeros_like(a)
    xh = np.zeros_like(a)
    act = _load().tor_prox_vel(pa, pb, _w(wl), _w(wh), float(C), a.shape[0], int(bool(minimum)),
                               xl.ctypes.data_as(_dp), xh.ctypes.data_as(_dp))
    return bool(act), xl, xh


def prox_capsule(xL, xR, r, n0, n1, w0, w1):
    """Agent-wall minimiser, App. D/I.  Returns (active, x0, x1, kind, theta).

    kind: -1 inactive, 0 tangent slab, 1 boundary with x1 = n1, 2 boundary with x0 = n0."""
    arrs = [_d(v) for v in (xL, xR, n0, n1)]
    x0 = np.zeros(2)
    x1 = np.zeros(2)
    kind = ct.c_int(0)
    th = ct.c_double(0)
    act = _load().tor_prox_capsule(arrs[0][1], arrs[1][1], float(r), arrs[2][1], arrs[3][1], _w(w0), _w(w1),
                                   x0.ctypes.data_as(_dp), x1.ctypes.data_as(_dp), ct.byref(kind), ct.byref(th))
    return bool(act), x0, x1, kind.value, th.value


def prox_coll(nl, nh, nlp, nhp, wl, wh, wlp, whp, R):
    """Agent-agent minimiser, eq. coll_minimizer_problem via App. C.

    Returns (active, xl, xh, xlp, xhp, kind, theta)."""
    arrs = [_d(v) for v in (nl, nh, nlp, nhp)]
    dim = arrs[0][0].shape[0]
    outs = [np.zeros(dim) for _ in range(4)]
    kind = ct.c_int(0)
    th = ct.c_double(0)
    act = _load().tor_prox_coll(*[a[1] for a in arrs], _w(wl), _w(wh), _w(wlp), _w(whp), float(R), dim,
                                *[o.ctypes.data_as(_dp) for o in outs], ct.byref(kind), ct.byref(th))
    return (bool(act), *outs, kind.value, th.value)


def prox_capsule_gap(xL, xR, r, n0, n1, w0, w1) -> float:
    """Relative energy gap between the agent-wall minimiser's chosen
    configuration and the best distinct runner-up candidate (inf when the
    factor is inactive or has a single candidate): a near-tie diagnostic."""
    arrs = [_d(v) for v in (xL, xR, n0, n1)]
    x0 = np.zeros(2)
    x1 = np.zeros(2)
    kind = ct.c_int(0)
    th = ct.c_double(0)
    gap = ct.c_double(0)
    _load().tor_prox_capsule_gap(arrs[0][1], arrs[1][1], float(r), arrs[2][1], arrs[3][1], _w(w0), _w(w1),
                                 x0.ctypes.data_as(_dp), x1.ctypes.data_as(_dp), ct.byref(kind), ct.byref(th),
                                 ct.byref(gap))
    return gap.value


def prox_coll_gap(nl, nh, nlp, nhp, wl, wh, wlp, whp, R) -> float:
    """As prox_capsule_gap, for the agent-agent minimiser."""
    arrs = [_d(v) for v in (nl, nh, nlp, nhp)]
    dim = arrs[0][0].shape[0]
    outs = [np.zeros(dim) for _ in range(4)]
    kind = ct.c_int(0)
    th = ct.c_double(0)
    gap = ct.c_double(0)
    _load().tor_prox_coll_gap(*[a[1] for a in arrs], _w(wl), _w(wh), _w(wlp), _w(whp), float(R), dim,
                              *[o.ctypes.data_as(_dp) for o in outs], ct.byref(kind), ct.byref(th), ct.byref(gap))
    return gap.value


def min_clearance(radii, z, walls=None) -> float:
    """min over segment pairs of (closest approach - r_i - r_j) and over
    segment/wall pairs of (distance - r_i); z is [p][eta+1][dim]."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    p, E1, dim = z.shape
    r, pr = _d(radii)
    if walls is None or len(walls) == 0:
        wa, pw, W = None, None, 0
    else:
        wa, pw = _d(np.asarray(walls).reshape(-1, 4))
        W = wa.shape[0]
    return _load().tor_min_clearance(p, E1 - 1, dim, pr, z.ctypes.data_as(_dp), W, pw)


# ------------------------------------------------------------------ planner

class Planner:
    """The full planner (App. B) on one instance, in FP64."""

    def __init__(self, inst, mode: int = MODE_TWA, cost: int = COST_ENERGY):
        lib = _load()
        self.inst = inst
        self.p, self.eta, self.dim = inst.p, inst.eta, inst.dim
        self._keep = [_d(inst.radii), _d(inst.x0), _d(inst.xT), _d(np.asarray(inst.walls).reshape(-1, 4)
                      if inst.n_walls else np.zeros(4)), _d(inst.C)]
        self.h = lib.tor_create(inst.p, inst.eta, inst.dim, self._keep[0][1], self._keep[1][1],
                                self._keep[2][1], inst.n_walls, self._keep[3][1], self._keep[4][1],
                                float(inst.rho0), float(inst.alpha), int(mode), int(cost))
        if not self.h:
            raise ValueError("invalid instance for the reference planner")
        self.F = lib.tor_num_factors(self.h)
        self.E = lib.tor_num_edges(self.h)
        self.N = (self.eta + 1) * self.p
        # initial state: z0 from the instance, u = 0, default <-rho
        lrho = np.full((self.p, self.eta + 1), INF if mode == MODE_TWA else STD, dtype=np.uint8)
        if self.eta > 1:
            lrho[:, 1:self.eta] = STD
        if cost == COST_VO:
            lrho[:, self.eta] = STD  # the reference end is soft
        self.set_state(inst.z0, np.zeros((self.E, self.dim)), lrho, 0)

    def __del__(self):
        if getattr(self, "h", None):
            _load().tor_destroy(self.h)
            self.h = None

    def set_schedule(self, rho0_init: float, n_warm: int):
        _load().tor_set_schedule(self.h, float(rho0_init), int(n_warm))

    def set_state(self, z, u, lrho, k: int = 0):
        z = np.ascontiguousarray(z, dtype=np.float64).reshape(self.N, self.dim)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.E, self.dim)
        lr = np.ascontiguousarray(lrho, dtype=np.uint8).reshape(self.N)
        _load().tor_set_state(self.h, z.ctypes.data_as(_dp), u.ctypes.data_as(_dp), lr.ctypes.data_as(_u8), int(k))

    def get_state(self):
        z = np.zeros((self.N, self.dim))
        u = np.zeros((self.E, self.dim))
        lr = np.zeros(self.N, dtype=np.uint8)
        _load().tor_get_state(self.h, z.ctypes.data_as(_dp), u.ctypes.data_as(_dp), lr.ctypes.data_as(_u8))
        return z.reshape(self.p, self.eta + 1, self.dim), u, lr.reshape(self.p, self.eta + 1)

    def last(self):
        """x per edge and ->rho per factor of the last iteration."""
        x = np.zeros((self.E, self.dim))
        rf = np.zeros(self.F, dtype=np.uint8)
        _load().tor_get_last(self.h, x.ctypes.data_as(_dp), rf.ctypes.data_as(_u8))
        return x, rf

    def margins(self):
        """Per-factor near-tie diagnostics of the last iteration:
        |closest approach - R|/R of the activity test, and the relative energy
        gap between the chosen candidate and the best distinct runner-up."""
        a = np.zeros(self.F)
        t = np.zeros(self.F)
        _load().tor_get_margins(self.h, a.ctypes.data_as(_dp), t.ctypes.data_as(_dp))
        return a, t

    def iterate(self, k: int):
        _load().tor_iterate(self.h, int(k))

    def override_next(self, factors, x, rho):
        """Test support: in the next iteration only, the listed factors emit
        the given x (their edges in canonical order, factors in the listed
        order) and ->rho instead of running their minimiser."""
        f = np.ascontiguousarray(factors, dtype=np.int64).ravel()
        xx = np.ascontiguousarray(x, dtype=np.float64).ravel()
        rr = np.ascontiguousarray(rho, dtype=np.uint8).ravel()
        if f.size == 0:
            return
        _load().tor_override_next(self.h, int(f.size), f.ctypes.data_as(ct.POINTER(ct.c_long)),
                                  xx.ctypes.data_as(_dp), rr.ctypes.data_as(_u8))

    def tape(self, k: int):
        """Run k iterations keeping every state for :meth:`backward`."""
        got = _load().tor_tape(self.h, int(k))
        if got == -2:
            raise ValueError("the reference adjoint covers the energy cost only")
        if got != k:
            raise MemoryError("tape allocation failed")

    def backward(self, dz):
        """Gradient of L(z^K) after :meth:`tape`, given dL/dz^K [p][eta+1][dim]:
        returns (dx0 [p][dim], dxT [p][dim], dr [p], dz0 [p][eta+1][dim], interior only)."""
        dz = np.ascontiguousarray(dz, dtype=np.float64).reshape(self.N, self.dim)
        dx0 = np.zeros((self.p, self.dim))
        dxT = np.zeros((self.p, self.dim))
        dr = np.zeros(self.p)
        dz0 = np.zeros((self.N, self.dim))
        _load().tor_backward(self.h, dz.ctypes.data_as(_dp), dx0.ctypes.data_as(_dp), dxT.ctypes.data_as(_dp),
                             dr.ctypes.data_as(_dp), dz0.ctypes.data_as(_dp))
        return dx0, dxT, dr, dz0.reshape(self.p, self.eta + 1, self.dim)

    @property
    def iteration(self) -> int:
        return _load().tor_iteration(self.h)

    def trajectories(self):
        return self.get_state()[0]

    def objective(self) -> float:
        return _load().tor_objective(self.h)

    def min_clearance(self) -> float:
        return min_clearance(self.inst.radii, self.trajectories(), self.inst.walls)
