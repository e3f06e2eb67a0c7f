"""The HIP library's FP32 minimisers (prox.h), compiled for the host, agree
case by case with the FP64 reference minimisers (no GPU).

Inputs are rounded to FP32 first; cases whose two best candidate
configurations are within 1e-5 in energy (near-ties, where FP32 and FP64
may choose differently) are counted and skipped.
"""
import ctypes as ct
import os
import zlib
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
from oracle.ref import _dp, _ip, _load
from tests import bruteforce as bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOL = 1e-5
_fp = ct.POINTER(ct.c_float)
_i32 = ct.POINTER(ct.c_int)


@pytest.fixture(scope="module")
def H():
    d = tempfile.mkdtemp(prefix="twa_host_")
    so = os.path.join(d, "libhost_prox.so")
    subprocess.run(["hipcc", "-O2", "-fPIC", "-shared", "-std=c++17", "-o", so,
                    os.path.join(ROOT, "tests", "host_prox.cpp")], check=True)
    lib = ct.CDLL(so)
    lib.h_coll.argtypes = [ct.c_int, _fp, _fp, _i32, ct.c_float, _fp]
    lib.h_capsule.argtypes = [_fp, ct.c_float, _fp, ct.c_float, ct.c_float, ct.c_int, ct.c_int, _fp]
    lib.h_energy.argtypes = [_fp, _fp, ct.c_int, ct.c_float, ct.c_float, ct.c_int, ct.c_int, ct.c_float, _fp, _fp]
    return lib


def _ref_lib():
    L = _load()
    L.tor_prox_capsule_gap.restype = ct.c_int
    L.tor_prox_capsule_gap.argtypes = [_dp, _dp, ct.c_double, _dp, _dp, ct.c_double, ct.c_double, _dp, _dp, _ip,
                                       _dp, _dp]
    L.tor_prox_coll_gap.restype = ct.c_int
    L.tor_prox_coll_gap.argtypes = [_dp, _dp, _dp, _dp, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                    ct.c_double, ct.c_int, _dp, _dp, _dp, _dp, _ip, _dp, _dp]
    return L


def _seed(*key):
    """A fixed seed per parametrisation (hash() of strings changes per process)."""
    return zlib.crc32(repr(key).encode())


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def _d(a):
    return np.ascontiguousarray(np.asarray(a, np.float64))


def ref_coll(n, w, R):
    L = _ref_lib()
    dim = n.shape[1]
    nn = [_d(v) for v in n]
    xs = [np.zeros(dim) for _ in range(4)]
    k, th, g = ct.c_int(), ct.c_double(), ct.c_double()
    act = L.tor_prox_coll_gap(*[v.ctypes.data_as(_dp) for v in nn], *[float(x) for x in w], float(R), dim,
                              *[x.ctypes.data_as(_dp) for x in xs], ct.byref(k), ct.byref(th), ct.byref(g))
    return bool(act), np.concatenate(xs), g.value


def ref_capsule(a, b, r, n0, n1, w0, w1):
    L = _ref_lib()
    arrs = [_d(v) for v in (a, b, n0, n1)]
    x0, x1 = np.zeros(2), np.zeros(2)
    k, th, g = ct.c_int(), ct.c_double(), ct.c_double()
    act = L.tor_prox_capsule_gap(arrs[0].ctypes.data_as(_dp), arrs[1].ctypes.data_as(_dp), float(r),
                                 arrs[2].ctypes.data_as(_dp), arrs[3].ctypes.data_as(_dp), float(w0), float(w1),
                                 x0.ctypes.data_as(_dp), x1.ctypes.data_as(_dp), ct.byref(k), ct.byref(th),
                                 ct.byref(g))
    return bool(act), np.concatenate([x0, x1]), g.value


def _close(a, b):
    return np.all(np.abs(a - b) <= TOL * np.maximum(np.abs(b), 1.0))


def _sensitivity(fn, v, ref, draws=16):
    """Largest change of fn's FP64 answer when every input moves by up to
    one FP32 unit in the last place (relative 2^-24), over seeded draws."""
    rng = np.random.default_rng(1)
    return max(np.abs(fn(v * (1 + rng.uniform(-1, 1, v.shape) * 2.0 ** -24)) - ref).max() for _ in range(draws))


WEIGHTS = {"std": ([1.0] * 4, [1] * 4), "inf_lo": ([0.0, 1.0, 0.0, 1.0], [2, 1, 2, 1]),
           "inf_hi": ([1.0, 0.0, 1.0, 0.0], [1, 2, 1, 2]), "unequal": (None, [1] * 4)}


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("wmode", list(WEIGHTS))
@pytest.mark.parametrize("scale", [1.0, 0.01])
def test_coll_matches_reference(H, dim, wmode, scale):
    rng = np.random.default_rng(_seed(dim, wmode, scale))
    R = 0.5 * scale
    checked = ties = conditioned = 0
    for _ in range(3000):
        n = _f32(rng.normal(0, 0.4 * scale, size=(4, dim))).astype(np.float64)
        w, k = WEIGHTS[wmode]
        if w is None:
            w = list(rng.uniform(0.3, 3.0, size=4))
        if wmode != "std" and wmode != "unequal":
            fixed = (0, 2) if wmode == "inf_lo" else (1, 3)
            if np.linalg.norm(n[fixed[1]] - n[fixed[0]]) < R * 1.001:
                continue
        wref = [np.inf if kk == 2 else ww for ww, kk in zip(w, k)]
        act, xr, gap = ref_coll(n, wref, R)
        if not act:
            continue
        if gap < TOL:
            ties += 1
            continue
        x = np.zeros(4 * dim, np.float32)
        H.h_coll(dim, _f32(n.reshape(-1)).ctypes.data_as(_fp), _f32(w).ctypes.data_as(_fp),
                 np.ascontiguousarray(k, np.int32).ctypes.data_as(_i32), R, x.ctypes.data_as(_fp))
        ok = _close(x.astype(np.float64), xr)
        if not ok:
            # an ill-conditioned case: the FP32 minimiser rounds its inputs
            # and a handful of intermediates, each about one unit in the last
            # place, so it may differ by several times what one such
            # perturbation of the inputs moves the FP64 answer by (8 allowed)
            dev = _sensitivity(lambda m: ref_coll(m, wref, R)[1], n, xr)
            ok = np.abs(x - xr).max() <= 8 * dev
            conditioned += 1
        assert ok, (n, w, k, x, xr)
        checked += 1
        if checked >= 300:
            break
    assert checked >= 100 and ties <= 0.02 * checked and conditioned <= 0.01 * checked


@pytest.mark.parametrize("wmode", ["std", "inf0", "inf1", "unequal"])
@pytest.mark.parametrize("scale", [1.0, 0.02])
def test_capsule_matches_reference(H, wmode, scale):
    rng = np.random.default_rng(_seed(wmode, scale))
    checked = ties = 0
    for _ in range(4000):
        r = float(np.float32(rng.uniform(0.05, 0.3) * scale))
        c = rng.uniform(-0.3, 0.3, 2) * scale
        th = rng.uniform(0, np.pi)
        L = rng.uniform(0, 0.8) * scale
        h = 0.5 * L * np.array([np.cos(th), np.sin(th)])
        a, b = _f32(c - h).astype(np.float64), _f32(c + h).astype(np.float64)
        n = _f32(rng.normal(0, 0.4 * scale, 4)).astype(np.float64)
        w0, w1 = (rng.uniform(0.3, 3.0, 2) if wmode == "unequal" else (1.0, 1.0))
        k0 = 2 if wmode == "inf0" else 1
        k1 = 2 if wmode == "inf1" else 1
        if k0 == 2 and bf.point_seg(n[:2], a, b) < r * 1.001:
            continue
        if k1 == 2 and bf.point_seg(n[2:], a, b) < r * 1.001:
            continue
        act, xr, gap = ref_capsule(a, b, r, n[:2], n[2:], np.inf if k0 == 2 else w0, np.inf if k1 == 2 else w1)
        if not act:
            continue
        if gap < TOL:
            ties += 1
            continue
        x = np.zeros(4, np.float32)
        H.h_capsule(_f32(np.concatenate([a, b])).ctypes.data_as(_fp), r, _f32(n).ctypes.data_as(_fp), float(w0),
                    float(w1), k0, k1, x.ctypes.data_as(_fp))
        assert _close(x.astype(np.float64), xr), (a, b, r, n, w0, w1, k0, k1, x, xr)
        checked += 1
        if checked >= 300:
            break
    assert checked >= 100 and ties <= 0.02 * checked


def test_energy_matches_reference(H):
    rng = np.random.default_rng(5)
    for _ in range(200):
        nl, nh = _f32(rng.normal(size=3)), _f32(rng.normal(size=3))
        wl, wh, C = (float(np.float32(v)) for v in rng.uniform(0.05, 3, 3))
        for kl, kh in [(1, 1), (2, 1), (1, 2), (2, 2)]:
            xl, xh = np.zeros(3, np.float32), np.zeros(3, np.float32)
            H.h_energy(nl.ctypes.data_as(_fp), nh.ctypes.data_as(_fp), 3, wl, wh, kl, kh, C, xl.ctypes.data_as(_fp),
                       xh.ctypes.data_as(_fp))
            rl, rh = O.prox_energy(nl, nh, np.inf if kl == 2 else wl, np.inf if kh == 2 else wh, C)
            assert _close(xl, rl) and _close(xh, rh)


# ------------------------------------------------------------------ derivatives

def _fd_vjp(fn, x, xb, h):
    """sum_o xb_o d fn_o / d x_q by FP64 central differences, for each q."""
    out = np.zeros(len(x))
    for q in range(len(x)):
        a, b = x.copy(), x.copy()
        a[q] += h
        b[q] -= h
        out[q] = np.dot((fn(a) - fn(b)) / (2 * h), xb)
    return out


def _vjp_close(g, want, tol=2e-4):
    return np.linalg.norm(g - want) <= tol * max(np.linalg.norm(want), 1e-3)


@pytest.mark.parametrize("wmode", list(WEIGHTS))
@pytest.mark.parametrize("scale", [1.0, 0.01])
def test_coll_vjp_matches_reference_differences(H, wmode, scale):
    H.h_coll_vjp.argtypes = [_fp, _fp, _i32, ct.c_float, _fp, _fp, _fp]
    rng = np.random.default_rng(_seed("vjp", wmode, scale))
    R = 0.5 * scale
    checked = 0
    for _ in range(4000):
        n = _f32(rng.normal(0, 0.4 * scale, size=(4, 2))).astype(np.float64)
        w, k = WEIGHTS[wmode]
        if w is None:
            w = list(rng.uniform(0.3, 3.0, size=4))
        if wmode in ("inf_lo", "inf_hi"):
            fixed = (0, 2) if wmode == "inf_lo" else (1, 3)
            if np.linalg.norm(n[fixed[1]] - n[fixed[0]]) < R * 1.01:
                continue
        wref = [np.inf if kk == 2 else ww for ww, kk in zip(w, k)]
        act, xr, gap = ref_coll(n, wref, R)
        if not act or gap < 1e-3:
            continue
        xb = rng.normal(size=8)
        vec = np.concatenate([n.reshape(-1), [R]])

        def fn(v):
            return ref_coll(v[:8].reshape(4, 2), wref, v[8])[1]
        fd1 = _fd_vjp(fn, vec, xb, 1e-6 * scale)
        fd2 = _fd_vjp(fn, vec, xb, 3e-7 * scale)
        if np.linalg.norm(fd1 - fd2) > 1e-5 * max(np.linalg.norm(fd1), 1.0):
            continue  # a branch switch within the step
        nb = np.zeros(8, np.float32)
        Rb = np.zeros(1, np.float32)
        H.h_coll_vjp(_f32(n.reshape(-1)).ctypes.data_as(_fp), _f32(w).ctypes.data_as(_fp),
                     np.ascontiguousarray(k, np.int32).ctypes.data_as(_i32), R, _f32(xb).ctypes.data_as(_fp),
                     nb.ctypes.data_as(_fp), Rb.ctypes.data_as(_fp))
        got = np.concatenate([nb, Rb]).astype(np.float64)
        assert _vjp_close(got, fd1), (n, w, k, got, fd1)
        checked += 1
        if checked >= 150:
            break
    assert checked >= 60


@pytest.mark.parametrize("wmode", ["std", "inf0", "inf1", "unequal"])
def test_capsule_vjp_matches_reference_differences(H, wmode):
    H.h_capsule_vjp.argtypes = [_fp, ct.c_float, _fp, ct.c_float, ct.c_float, ct.c_int, ct.c_int, _fp, _fp, _fp]
    rng = np.random.default_rng(_seed("cvjp", wmode))
    checked = 0
    for _ in range(6000):
        r = float(np.float32(rng.uniform(0.05, 0.3)))
        c = rng.uniform(-0.3, 0.3, 2)
        th = rng.uniform(0, np.pi)
        L = rng.uniform(0, 0.8)
        hh = 0.5 * L * np.array([np.cos(th), np.sin(th)])
        a, b = _f32(c - hh).astype(np.float64), _f32(c + hh).astype(np.float64)
        n = _f32(rng.normal(0, 0.4, 4)).astype(np.float64)
        w0, w1 = (rng.uniform(0.3, 3.0, 2) if wmode == "unequal" else (1.0, 1.0))
        k0 = 2 if wmode == "inf0" else 1
        k1 = 2 if wmode == "inf1" else 1
        if k0 == 2 and bf.point_seg(n[:2], a, b) < r * 1.01:
            continue
        if k1 == 2 and bf.point_seg(n[2:], a, b) < r * 1.01:
            continue
        W0, W1 = (np.inf if k0 == 2 else w0), (np.inf if k1 == 2 else w1)
        act, xr, gap = ref_capsule(a, b, r, n[:2], n[2:], W0, W1)
        if not act or gap < 1e-3:
            continue
        xb = rng.normal(size=4)
        vec = np.concatenate([n, [r]])

        def fn(v):
            return ref_capsule(a, b, v[4], v[:2], v[2:4], W0, W1)[1]
        fd1 = _fd_vjp(fn, vec, xb, 1e-6)
        fd2 = _fd_vjp(fn, vec, xb, 3e-7)
        if np.linalg.norm(fd1 - fd2) > 1e-5 * max(np.linalg.norm(fd1), 1.0):
            continue
        nb = np.zeros(4, np.float32)
        rb = np.zeros(1, np.float32)
        H.h_capsule_vjp(_f32(np.concatenate([a, b])).ctypes.data_as(_fp), r, _f32(n).ctypes.data_as(_fp),
                        float(w0), float(w1), k0, k1, _f32(xb).ctypes.data_as(_fp), nb.ctypes.data_as(_fp),
                        rb.ctypes.data_as(_fp))
        got = np.concatenate([nb, rb]).astype(np.float64)
        assert _vjp_close(got, fd1), (a, b, r, n, w0, w1, k0, k1, got, fd1)
        checked += 1
        if checked >= 150:
            break
    assert checked >= 60


def test_energy_vjp_matches_reference_differences(H):
    H.h_energy_vjp.argtypes = [ct.c_float, ct.c_float, ct.c_int, ct.c_int, ct.c_float, ct.c_float, ct.c_float, _fp,
                               _fp]
    rng = np.random.default_rng(17)
    for _ in range(100):
        wl, wh, C = (float(np.float32(v)) for v in rng.uniform(0.05, 3, 3))
        xlb, xhb = rng.normal(size=2)
        for kl, kh in [(1, 1), (2, 1), (1, 2)]:
            Wl, Wh = (np.inf if kl == 2 else wl), (np.inf if kh == 2 else wh)

            def fn(v):
                a, b = O.prox_energy([v[0]], [v[1]], Wl, Wh, C)
                return np.array([a[0], b[0]])
            fd = _fd_vjp(fn, np.array([0.3, -0.2]), np.array([xlb, xhb]), 1e-6)
            a = np.zeros(1, np.float32)
            b = np.zeros(1, np.float32)
            H.h_energy_vjp(wl, wh, kl, kh, C, xlb, xhb, a.ctypes.data_as(_fp), b.ctypes.data_as(_fp))
            assert np.allclose([a[0], b[0]], fd, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("ratio", [0.5, 0.9, -0.4])
def test_coll_vjp_parallel_differences(H, ratio):
    """Both relative positions on one line through the origin and inside the
    disk (agents heading straight at each other, the straight-line start of a
    circle swap): the minimiser is the tangent-family stationary point, whose
    derivative the VJP must give (a radial push of one end alone would be a
    tie in value but not in derivative)."""
    H.h_coll_vjp.argtypes = [_fp, _fp, _i32, ct.c_float, _fp, _fp, _fp]
    rng = np.random.default_rng(int(1000 * (ratio + 1)))
    R = 0.6
    checked = 0
    for _ in range(200):
        d = rng.normal(size=2)
        d /= np.linalg.norm(d)
        a = rng.uniform(0.05, 0.5)
        base = rng.normal(0, 0.3, size=(2, 2))
        m0, m1 = a * d, ratio * a * d + rng.normal(0, 1e-4, size=2)
        n = np.array([base[0], base[1], base[0] + m0, base[1] + m1])
        n = _f32(n).astype(np.float64)
        act, xr, gap = ref_coll(n, [1.0] * 4, R)
        if not act or gap < 1e-3:
            continue
        xb = rng.normal(size=8)
        vec = np.concatenate([n.reshape(-1), [R]])

        def fn(v):
            return ref_coll(v[:8].reshape(4, 2), [1.0] * 4, v[8])[1]
        fd1 = _fd_vjp(fn, vec, xb, 1e-9)
        fd2 = _fd_vjp(fn, vec, xb, 1e-8)
        if np.linalg.norm(fd1 - fd2) > 1e-4 * max(np.linalg.norm(fd1), 1.0):
            continue
        nb = np.zeros(8, np.float32)
        Rb = np.zeros(1, np.float32)
        H.h_coll_vjp(_f32(n.reshape(-1)).ctypes.data_as(_fp), _f32([1.0] * 4).ctypes.data_as(_fp),
                     np.ones(4, np.int32).ctypes.data_as(_i32), R, _f32(xb).ctypes.data_as(_fp),
                     nb.ctypes.data_as(_fp), Rb.ctypes.data_as(_fp))
        got = np.concatenate([nb, Rb]).astype(np.float64)
        assert _vjp_close(got, fd1), (n, got, fd1)
        checked += 1
        if checked >= 40:
            break
    assert checked >= 20


@pytest.mark.parametrize("minimum", [False, True])
@pytest.mark.parametrize("wmode", ["std", "inf_lo", "inf_hi", "unequal"])
def test_velocity_minimiser_matches_reference(H, minimum, wmode):
    H.h_vel.argtypes = [ct.c_int, _fp, _fp, ct.c_float, ct.c_float, ct.c_int, ct.c_int, ct.c_float, ct.c_int, _fp,
                        _fp]
    H.h_vel.restype = ct.c_int
    rng = np.random.default_rng(_seed("vel", minimum, wmode))
    for _ in range(300):
        dim = int(rng.choice([2, 3]))
        nl = _f32(rng.normal(0, 1, dim)).astype(np.float64)
        nh = _f32(rng.normal(0, 1, dim)).astype(np.float64)
        C = float(np.float32(rng.uniform(0.2, 2.5)))
        d = np.linalg.norm(nl - nh)
        if abs(d - C) < 1e-4 * C:
            continue  # the binding test itself is within rounding
        wl, wh = (float(np.float32(v)) for v in rng.uniform(0.2, 3.0, 2))
        if wmode == "std":
            wl = wh = 1.0
        kl = 2 if wmode == "inf_lo" else 1
        kh = 2 if wmode == "inf_hi" else 1
        act, xl, xh = O.prox_vel(nl, nh, np.inf if kl == 2 else wl, np.inf if kh == 2 else wh, C, minimum)
        gl = np.zeros(dim, np.float32)
        gh = np.zeros(dim, np.float32)
        got = H.h_vel(dim, _f32(nl).ctypes.data_as(_fp), _f32(nh).ctypes.data_as(_fp), wl, wh, kl, kh, C,
                      int(minimum), gl.ctypes.data_as(_fp), gh.ctypes.data_as(_fp))
        assert bool(got) == act
        assert _close(np.concatenate([gl, gh]).astype(np.float64), np.concatenate([xl, xh]))
