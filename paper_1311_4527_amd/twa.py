"""Python binding of the C ABI in ``include/twa.h`` (argument marshalling only).

Every function of the library is exposed under the same name; ``Solver``
wraps a ``twa_solver*`` and owns it.  PyTorch provides the device memory
(CUDA tensors on the HIP device; the solvers' own buffers come from torch's
caching allocator through ``twa_set_allocator``) and the stream.  Every step
of the planner runs in the HIP kernels of ``libtwa.so``: if the library is
missing this module raises, there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as ct
import os
import weakref
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtwa.so")

TWA_OK, TWA_E_INVALID, TWA_E_INFEASIBLE, TWA_E_NOMEM, TWA_E_DEVICE, TWA_E_NUMERIC, TWA_E_STATE = range(7)
TWA_W_ZERO, TWA_W_STD, TWA_W_INF = 0, 1, 2
TWA_F_DENSE = 1
TWA_F_TAPE = 2
TWA_F_ADMM = 4
TWA_F_COST_NONE = 8
TWA_F_COST_MAXVEL = 16
TWA_F_COST_MINVEL = 32
TWA_F_VO = 64
_STATUS = {0: "TWA_OK", 1: "TWA_E_INVALID", 2: "TWA_E_INFEASIBLE", 3: "TWA_E_NOMEM", 4: "TWA_E_DEVICE",
           5: "TWA_E_NUMERIC", 6: "TWA_E_STATE"}


class TWAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Stats(ct.Structure):
    _fields_ = [("iter", ct.c_longlong), ("active_coll", ct.c_longlong), ("active_wall", ct.c_longlong),
                ("queued", ct.c_longlong), ("residual", ct.c_double), ("objective", ct.c_double),
                ("min_clearance", ct.c_double), ("graph_iterations", ct.c_longlong),
                ("tape_checkpoints", ct.c_longlong)]


_lib = None
_vp = ct.c_void_p
_ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_int, ct.c_void_p, ct.c_void_p)
_FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_size_t, ct.c_int, ct.c_void_p, ct.c_void_p)
_live = weakref.WeakSet()   # solvers and batches that own library objects


def _torch_alloc(nbytes, device, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device), stream=int(stream or 0))
    except Exception:  # NULL: the library call fails with TWA_E_NOMEM
        return None


def _torch_free(ptr, nbytes, device, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept alive for as long as the library may call them
_torch_alloc_c = _ALLOC_FN(_torch_alloc)
_torch_free_c = _FREE_FN(_torch_free)


def twa_set_allocator(use_torch: bool = True):
    """Where solvers and batches created from now on take their device
    buffers: torch's caching allocator (the default, set when the library
    is loaded) or plain hipMalloc/hipFree (use_torch=False)."""
    lib = load_library()
    if use_torch:
        st = lib.twa_set_allocator(_torch_alloc_c, _torch_free_c, None)
    else:
        st = lib.twa_set_allocator(_ALLOC_FN(), _FREE_FN(), None)
    if st != TWA_OK:
        raise TWAError(st, "twa_set_allocator failed")


@atexit.register
def _close_all():
    # destroy what is still alive while torch's allocator can take the
    # memory back (before the interpreter tears the modules down)
    for o in list(_live):
        try:
            o.close()
        except Exception:
            pass


def load_library():
    """Load ``libtwa.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1311_4527_amd/build.py")
    lib = ct.CDLL(LIB_PATH)
    lib.twa_create.restype = ct.c_int
    lib.twa_create.argtypes = [ct.c_int, ct.c_int, ct.c_int, _vp, _vp, _vp, ct.c_int, _vp, _vp, ct.c_float,
                               ct.c_float, ct.c_uint, _vp, ct.POINTER(_vp)]
    lib.twa_set_init.restype = ct.c_int
    lib.twa_set_init.argtypes = [_vp, _vp]
    lib.twa_set_endpoints.restype = ct.c_int
    lib.twa_set_endpoints.argtypes = [_vp, _vp, _vp]
    lib.twa_set_schedule.restype = ct.c_int
    lib.twa_set_schedule.argtypes = [_vp, ct.c_float, ct.c_int]
    lib.twa_iterate.restype = ct.c_int
    lib.twa_iterate.argtypes = [_vp, ct.c_int]
    lib.twa_iterate_until.restype = ct.c_int
    lib.twa_iterate_until.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_double, ct.POINTER(ct.c_int),
                                      ct.POINTER(ct.c_int)]
    lib.twa_iterate_timed.restype = ct.c_int
    lib.twa_iterate_timed.argtypes = [_vp, ct.c_int, ct.POINTER(ct.c_double)]
    lib.twa_get_trajectories.restype = ct.c_int
    lib.twa_get_trajectories.argtypes = [_vp, _vp]
    lib.twa_get_state.restype = ct.c_int
    lib.twa_get_state.argtypes = [_vp, _vp, _vp, _vp, ct.POINTER(ct.c_longlong)]
    lib.twa_set_state.restype = ct.c_int
    lib.twa_set_state.argtypes = [_vp, _vp, _vp, _vp, ct.c_longlong]
    lib.twa_capture_next.restype = ct.c_int
    lib.twa_capture_next.argtypes = [_vp, _vp, _vp]
    lib.twa_get_stats.restype = ct.c_int
    lib.twa_get_stats.argtypes = [_vp, ct.POINTER(_Stats)]
    lib.twa_sizes.restype = ct.c_int
    lib.twa_sizes.argtypes = [_vp, ct.POINTER(ct.c_longlong), ct.POINTER(ct.c_longlong)]
    lib.twa_get_quality.restype = ct.c_int
    lib.twa_get_quality.argtypes = [_vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
    lib.twa_check_finite.restype = ct.c_int
    lib.twa_check_finite.argtypes = [_vp]
    lib.twa_consensus_scale.restype = ct.c_int
    lib.twa_consensus_scale.argtypes = [ct.c_int, ct.c_int, ct.c_double, ct.POINTER(ct.c_double),
                                        ct.POINTER(ct.c_double)]
    lib.twa_backward.restype = ct.c_int
    lib.twa_backward.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    lib.twa_backward_noalloc.restype = ct.c_int
    lib.twa_backward_noalloc.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp]
    lib.twa_last_error.restype = ct.c_char_p
    lib.twa_last_error.argtypes = [_vp]
    lib.twa_destroy.restype = None
    lib.twa_destroy.argtypes = [_vp]
    lib.twa_version.restype = ct.c_char_p
    lib.twa_version.argtypes = []
    lib.twa_batch_create.restype = ct.c_int
    lib.twa_batch_create.argtypes = [ct.c_int, ct.c_void_p, ct.c_uint, _vp, ct.POINTER(_vp)]
    lib.twa_batch_config.restype = ct.c_int
    lib.twa_batch_config.argtypes = [_vp, ct.c_int, ct.c_int]
    lib.twa_batch_iterate.restype = ct.c_int
    lib.twa_batch_iterate.argtypes = [_vp, ct.c_int]
    lib.twa_batch_iterate_timed.restype = ct.c_int
    lib.twa_batch_iterate_timed.argtypes = [_vp, ct.c_int, ct.POINTER(ct.c_double)]
    lib.twa_batch_size.restype = ct.c_int
    lib.twa_batch_size.argtypes = [_vp, ct.POINTER(ct.c_int)]
    lib.twa_batch_solver.restype = ct.c_int
    lib.twa_batch_solver.argtypes = [_vp, ct.c_int, ct.POINTER(_vp)]
    lib.twa_batch_get_trajectories.restype = ct.c_int
    lib.twa_batch_get_trajectories.argtypes = [_vp, ct.c_int, _vp]
    lib.twa_batch_last_error.restype = ct.c_char_p
    lib.twa_batch_last_error.argtypes = [_vp]
    lib.twa_batch_destroy.restype = None
    lib.twa_batch_destroy.argtypes = [_vp]
    lib.twa_set_allocator.restype = ct.c_int
    lib.twa_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, _vp]
    if lib.twa_set_allocator(_torch_alloc_c, _torch_free_c, None) != TWA_OK:
        raise TWAError(TWA_E_INVALID, "twa_set_allocator failed")
    _lib = lib
    return lib


def _dev(a, dtype=torch.float32, device="cuda") -> torch.Tensor:
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.asarray(a), dtype=dtype, device=device)
    return t.contiguous()


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ct.c_void_p(t.data_ptr())


class Solver:
    """One planning problem on the GPU (twa_create ... twa_destroy)."""

    def __init__(self, p, eta, dim, radii, x0, xT, walls=None, C=None, rho0=1.0, alpha=1.0, flags=0,
                 stream: Optional[torch.cuda.Stream] = None, device="cuda"):
        lib = load_library()
        self.p, self.eta, self.dim = int(p), int(eta), int(dim)
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        nw = 0 if walls is None else int(np.asarray(walls).reshape(-1, 2, dim).shape[0]) if not isinstance(
            walls, torch.Tensor) else int(walls.reshape(-1, 2, dim).shape[0])
        if C is None:
            C = np.ones((p, eta))
        self._radii = _dev(radii, device=device)
        self._x0 = _dev(x0, device=device).reshape(p, dim)
        self._xT = _dev(xT, device=device).reshape(p, dim)
        self._walls = _dev(walls, device=device).reshape(nw, 2, dim) if nw else None
        self._C = _dev(C, device=device).reshape(p, eta)
        h = ct.c_void_p()
        with torch.cuda.stream(self.stream):
            st = lib.twa_create(self.p, self.eta, self.dim, _ptr(self._radii), _ptr(self._x0), _ptr(self._xT), nw,
                                _ptr(self._walls), _ptr(self._C), float(rho0), float(alpha), int(flags),
                                ct.c_void_p(self.stream.cuda_stream), ct.byref(h))
        if st != TWA_OK:
            raise TWAError(st, "twa_create failed")
        self.h = h
        _live.add(self)
        self.n_walls = nw
        nf, ne = ct.c_longlong(), ct.c_longlong()
        lib.twa_sizes(self.h, ct.byref(nf), ct.byref(ne))
        self.n_factors, self.n_edges = nf.value, ne.value

    @classmethod
    def from_instance(cls, inst, flags=0, stream=None, device="cuda", set_init=True):
        s = cls(inst.p, inst.eta, inst.dim, inst.radii, inst.x0, inst.xT,
                walls=inst.walls if inst.n_walls else None, C=inst.C, rho0=inst.rho0, alpha=inst.alpha,
                flags=flags, stream=stream, device=device)
        if set_init:
            s.twa_set_init(inst.z0)
        return s

    # -- error handling
    def _check(self, st):
        if st != TWA_OK:
            msg = load_library().twa_last_error(self.h)
            raise TWAError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            load_library().twa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, same names
    def twa_set_init(self, z):
        zt = _dev(z, device=self.device).reshape(self.p, self.eta + 1, self.dim)
        self._check(load_library().twa_set_init(self.h, _ptr(zt)))
        torch.cuda.current_stream(self.device).synchronize()

    def twa_set_endpoints(self, x0, xT):
        x0t = _dev(x0, device=self.device).reshape(self.p, self.dim)
        xTt = _dev(xT, device=self.device).reshape(self.p, self.dim)
        self._check(load_library().twa_set_endpoints(self.h, _ptr(x0t), _ptr(xTt)))

    def twa_set_schedule(self, rho0_init: float, n_warm: int):
        self._check(load_library().twa_set_schedule(self.h, float(rho0_init), int(n_warm)))

    def twa_iterate(self, k: int):
        self._check(load_library().twa_iterate(self.h, int(k)))

    def twa_iterate_until(self, max_iter: int, every: int, min_clearance: float):
        """Up to max_iter iterations in blocks of `every`, stopping after the
        first block whose smallest clearance is >= min_clearance; returns
        (iterations run, whether the bar was met)."""
        done, met = ct.c_int(), ct.c_int()
        self._check(load_library().twa_iterate_until(self.h, int(max_iter), int(every), float(min_clearance),
                                                     ct.byref(done), ct.byref(met)))
        return done.value, bool(met.value)

    def twa_iterate_timed(self, k: int):
        """k iterations with HIP events around each launch; returns the summed
        device milliseconds of (factor stream, queued minimisers, consensus)."""
        ms = (ct.c_double * 3)()
        self._check(load_library().twa_iterate_timed(self.h, int(k), ms))
        return list(ms)

    def twa_get_trajectories(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.p, self.eta + 1, self.dim), dtype=torch.float32, device=self.device)
        self._check(load_library().twa_get_trajectories(self.h, _ptr(out)))
        return out

    def twa_get_state(self):
        z = torch.empty((self.p, self.eta + 1, self.dim), dtype=torch.float32, device=self.device)
        u = torch.empty((self.n_edges, self.dim), dtype=torch.float32, device=self.device)
        lr = torch.empty((self.p, self.eta + 1), dtype=torch.uint8, device=self.device)
        it = ct.c_longlong()
        self._check(load_library().twa_get_state(self.h, _ptr(z), _ptr(u), _ptr(lr), ct.byref(it)))
        return z, u, lr, it.value

    def twa_set_state(self, z, u, lrho, iteration: int = 0):
        zt = _dev(z, device=self.device).reshape(self.p, self.eta + 1, self.dim)
        ut = _dev(u, device=self.device).reshape(self.n_edges, self.dim)
        lt = _dev(lrho, dtype=torch.uint8, device=self.device).reshape(self.p, self.eta + 1)
        self._check(load_library().twa_set_state(self.h, _ptr(zt), _ptr(ut), _ptr(lt), int(iteration)))
        self.stream.synchronize()

    def twa_capture_next(self, x_out: Optional[torch.Tensor], rho_out: Optional[torch.Tensor]):
        self._keep_dbg = (x_out, rho_out)
        self._check(load_library().twa_capture_next(self.h, _ptr(x_out), _ptr(rho_out)))

    def twa_get_stats(self) -> dict:
        s = _Stats()
        self._check(load_library().twa_get_stats(self.h, ct.byref(s)))
        return dict(iter=s.iter, active_coll=s.active_coll, active_wall=s.active_wall, queued=s.queued,
                    residual=s.residual, objective=s.objective, min_clearance=s.min_clearance,
                    graph_iterations=s.graph_iterations, tape_checkpoints=s.tape_checkpoints)

    def twa_get_quality(self) -> dict:
        """Energy objective, smallest clearance and largest last move of the
        current break-points, computed on the device (synchronises)."""
        o, c, m = ct.c_double(), ct.c_double(), ct.c_double()
        self._check(load_library().twa_get_quality(self.h, ct.byref(o), ct.byref(c), ct.byref(m)))
        return dict(objective=o.value, min_clearance=c.value, max_move=m.value)

    def twa_check_finite(self):
        self._check(load_library().twa_check_finite(self.h))

    def twa_backward(self, dL_dz, want_dz0: bool = True):
        """Gradient of L(z^K) for the run since the last create / set_init /
        set_state (solver created with TWA_F_TAPE): returns (dL/dx0 [p][dim],
        dL/dxT [p][dim], dL/dr [p], dL/dz0 [p][eta+1][dim] or None)."""
        dz = _dev(dL_dz, device=self.device).reshape(self.p, self.eta + 1, self.dim)
        dx0 = torch.empty((self.p, self.dim), dtype=torch.float32, device=self.device)
        dxT = torch.empty_like(dx0)
        dr = torch.empty((self.p,), dtype=torch.float32, device=self.device)
        dz0 = torch.empty_like(dz) if want_dz0 else None
        self._check(load_library().twa_backward(self.h, _ptr(dz), _ptr(dx0), _ptr(dxT), _ptr(dr), _ptr(dz0)))
        return dx0, dxT, dr, dz0

    def twa_backward_noalloc(self, dL_dz, dx0, dxT, dr, dz0=None):
        """twa_backward into caller-provided device tensors, with the library's
        static scratch instead of any allocation (see the header)."""
        self._check(load_library().twa_backward_noalloc(self.h, _ptr(dL_dz), _ptr(dx0), _ptr(dxT), _ptr(dr),
                                                        _ptr(dz0)))

    # -- convenience
    def step_debug(self):
        """One iteration that also returns x [E][dim] and ->rho per factor."""
        x = torch.empty((self.n_edges, self.dim), dtype=torch.float32, device=self.device)
        r = torch.empty((self.n_factors,), dtype=torch.uint8, device=self.device)
        self.twa_capture_next(x, r)
        self.twa_iterate(1)
        self.stream.synchronize()
        self._keep_dbg = None
        return x, r


class _Instance(ct.Structure):
    _fields_ = [("p", ct.c_int), ("eta", ct.c_int), ("dim", ct.c_int), ("n_walls", ct.c_int),
                ("radii", _vp), ("x0", _vp), ("xT", _vp), ("walls", _vp), ("C", _vp), ("z0", _vp),
                ("rho0", ct.c_float), ("alpha", ct.c_float)]


class _Borrowed(Solver):
    """A solver owned by a batch (never destroyed from Python)."""

    def __init__(self, h, inst, stream, device):
        self.h = h
        self.p, self.eta, self.dim = inst.p, inst.eta, inst.dim
        self.device = device
        self.stream = stream
        self.n_walls = inst.n_walls
        nf, ne = ct.c_longlong(), ct.c_longlong()
        load_library().twa_sizes(self.h, ct.byref(nf), ct.byref(ne))
        self.n_factors, self.n_edges = nf.value, ne.value

    def close(self):
        self.h = None


class Batch:
    """Many independent instances advanced together (twa_batch_create ...
    twa_batch_destroy): by one persistent launch, or by one launch per phase
    over all instances (twa_batch_config(0, 1))."""

    def __init__(self, instances, flags=0, stream: Optional[torch.cuda.Stream] = None, device="cuda"):
        lib = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.instances = list(instances)
        self._keep = []
        arr = (_Instance * len(self.instances))()
        for k, inst in enumerate(self.instances):
            t = dict(radii=_dev(inst.radii, device=device), x0=_dev(inst.x0, device=device),
                     xT=_dev(inst.xT, device=device), C=_dev(inst.C, device=device),
                     z0=_dev(inst.z0, device=device),
                     walls=_dev(inst.walls, device=device) if inst.n_walls else None)
            self._keep.append(t)
            arr[k] = _Instance(inst.p, inst.eta, inst.dim, inst.n_walls, _ptr(t["radii"]), _ptr(t["x0"]),
                               _ptr(t["xT"]), _ptr(t["walls"]), _ptr(t["C"]), _ptr(t["z0"]),
                               float(inst.rho0), float(inst.alpha))
        h = ct.c_void_p()
        st = lib.twa_batch_create(len(self.instances), ct.cast(arr, ct.c_void_p), int(flags),
                                  ct.c_void_p(self.stream.cuda_stream), ct.byref(h))
        if st != TWA_OK:
            raise TWAError(st, "twa_batch_create failed")
        self.h = h
        _live.add(self)
        self.stream.synchronize()

    def _check(self, st):
        if st != TWA_OK:
            msg = load_library().twa_batch_last_error(self.h)
            raise TWAError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            load_library().twa_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.instances)

    def twa_batch_config(self, block: int, groups: int):
        """block 256 / 512 / 1024 lanes with `groups` bins: the persistent
        kernel; block 0: the phased form (groups ignored)."""
        self._check(load_library().twa_batch_config(self.h, int(block), int(groups)))

    def twa_batch_iterate(self, k: int):
        self._check(load_library().twa_batch_iterate(self.h, int(k)))

    def twa_batch_iterate_timed(self, k: int) -> float:
        ms = ct.c_double()
        self._check(load_library().twa_batch_iterate_timed(self.h, int(k), ct.byref(ms)))
        return ms.value

    def twa_batch_size(self) -> int:
        n = ct.c_int()
        self._check(load_library().twa_batch_size(self.h, ct.byref(n)))
        return n.value

    def twa_batch_get_trajectories(self, i: int) -> torch.Tensor:
        inst = self.instances[i]
        out = torch.empty((inst.p, inst.eta + 1, inst.dim), dtype=torch.float32, device=self.device)
        self._check(load_library().twa_batch_get_trajectories(self.h, int(i), _ptr(out)))
        return out

    def twa_batch_solver(self, i: int) -> Solver:
        h = ct.c_void_p()
        self._check(load_library().twa_batch_solver(self.h, int(i), ct.byref(h)))
        return _Borrowed(h, self.instances[i], self.stream, self.device)


def twa_version() -> str:
    return load_library().twa_version().decode()


def twa_consensus_scale(p: int, n_walls: int, coord_max: float):
    """(scale, limit) of the fixed-point consensus sums twa_create picks
    (host only)."""
    sc, lim = ct.c_double(), ct.c_double()
    st = load_library().twa_consensus_scale(int(p), int(n_walls), float(coord_max), ct.byref(sc), ct.byref(lim))
    if st != TWA_OK:
        raise TWAError(st, "twa_consensus_scale")
    return sc.value, lim.value
