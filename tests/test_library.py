"""The C-ABI library loads and exports every symbol its header declares;
argument validation that needs no device (no GPU)."""
import ctypes as ct
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "twa.h")
LIB = os.path.join(ROOT, "paper_1311_4527_amd", "libtwa.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(twa_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1311_4527_amd.build import build
        build()
    return ct.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("twa_create", "twa_iterate", "twa_get_trajectories", "twa_get_state", "twa_set_state",
                 "twa_destroy", "twa_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(lib, n)


def test_version(lib):
    lib.twa_version.restype = ct.c_char_p
    assert lib.twa_version().decode().startswith("twa-mi355x")


@pytest.mark.parametrize("p,eta,dim,nw", [(0, 4, 2, 0), (4, 0, 2, 0), (4, 4, 4, 0), (4, 4, 3, 2), (4, 4, 2, -1)])
def test_create_rejects_bad_sizes_without_touching_the_device(lib, p, eta, dim, nw):
    lib.twa_create.restype = ct.c_int
    out = ct.c_void_p()
    dummy = ct.c_void_p(16)
    st = lib.twa_create(p, eta, dim, dummy, dummy, dummy, nw, dummy, dummy, ct.c_float(1.0), ct.c_float(1.0), 0,
                        None, ct.byref(out))
    assert st == 1 and not out.value


def test_create_rejects_bad_scalars(lib):
    lib.twa_create.restype = ct.c_int
    out = ct.c_void_p()
    dummy = ct.c_void_p(16)
    for rho, alpha, flags in [(0.0, 1.0, 0), (1.0, -1.0, 0), (float("nan"), 1.0, 0), (1.0, 1.0, 1 << 7)]:
        st = lib.twa_create(4, 4, 2, dummy, dummy, dummy, 0, None, dummy, ct.c_float(rho), ct.c_float(alpha), flags,
                            None, ct.byref(out))
        assert st == 1


@pytest.mark.parametrize("p,eta,nw", [(65537, 1, 0), (50000, 2, 0), (8, 1 << 16, 0), (4096, 16, 1 << 15),
                                       (4, 4, 1 << 24)])
def test_create_rejects_problems_past_the_index_range(lib, p, eta, nw):
    """Factor indices are 31-bit in the queues (collision or wall factors per
    kind < 2^31), break-point intervals < 2^16, walls < 2^24: larger problems
    are refused before any device work."""
    lib.twa_create.restype = ct.c_int
    lib.twa_last_error.restype = ct.c_char_p
    out = ct.c_void_p()
    dummy = ct.c_void_p(16)
    st = lib.twa_create(p, eta, 2, dummy, dummy, dummy, nw, dummy if nw else None, dummy, ct.c_float(1.0),
                        ct.c_float(0.1), 0, None, ct.byref(out))
    assert st == 1 and not out.value


def test_null_solver_calls(lib):
    lib.twa_iterate.restype = ct.c_int
    lib.twa_last_error.restype = ct.c_char_p
    assert lib.twa_iterate(None, 1) == 1
    lib.twa_destroy(None)
    assert lib.twa_last_error(None)


def test_binding_exposes_the_abi_names():
    from paper_1311_4527_amd import twa
    internal = ("twa_create", "twa_destroy", "twa_last_error", "twa_sizes", "twa_batch_create",
                "twa_batch_destroy", "twa_batch_last_error")
    for n in _declared():
        if n in internal:
            continue
        assert hasattr(twa.Solver, n) or hasattr(twa.Batch, n) or hasattr(twa, n), n


def test_create_rejects_flag_combinations(lib):
    lib.twa_create.restype = ct.c_int
    out = ct.c_void_p()
    dummy = ct.c_void_p(16)
    vo, none, maxv = 1 << 6, 1 << 3, 1 << 4
    for eta, flags in [(2, vo), (1, vo | none), (4, none | maxv)]:
        st = lib.twa_create(4, eta, 2, dummy, dummy, dummy, 0, None, dummy, ct.c_float(1.0), ct.c_float(0.1), flags,
                            None, ct.byref(out))
        assert st == 1 and not out.value


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures the one-GPU hot path; --gpus above 1 exits with
    a message instead of timing anything."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_traffic_digest_tracks_the_sources(tmp_path, monkeypatch):
    """Counter-based traffic is reported only for the kernel sources it was
    taken on: any change to the code (comments aside) turns it off."""
    import importlib
    import shutil
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    bench = importlib.import_module("bench")
    d = bench.kernel_sources_digest()
    for rel in bench.KERNEL_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(root, rel), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_sources_digest() == d
    p = tmp_path / bench.KERNEL_SOURCES[0]
    p.write_text(p.read_text() + "\n// a comment changes nothing\n")
    assert bench.kernel_sources_digest() == d
    p.write_text(p.read_text() + "\nstatic int twa_extra_symbol;\n")
    assert bench.kernel_sources_digest() != d
    for variant in bench.MEASURED_TRAFFIC:
        assert bench.measured_traffic(variant) is None


@pytest.mark.parametrize("p,nw,cmax", [(1, 0, 1.0), (8, 0, 1.0), (100, 0, 1.0), (1024, 32, 1.0), (4096, 4, 1.0),
                                       (64, 8, 37.5), (5000, 0, 1e6)])
def test_consensus_scale_headroom(lib, p, nw, cmax):
    """The fixed-point consensus: a power-of-two scale (at most 2^44) such that
    a node's degree of contributions, each within the overflow limit, sums
    below 2^62 (no int64 wrap), while every m of at most 8 coord_max -- far
    beyond any iterate that stays in the scene -- stays within the limit."""
    lib.twa_consensus_scale.restype = ct.c_int
    lib.twa_consensus_scale.argtypes = [ct.c_int, ct.c_int, ct.c_double, ct.POINTER(ct.c_double),
                                        ct.POINTER(ct.c_double)]
    sc, lim = ct.c_double(), ct.c_double()
    assert lib.twa_consensus_scale(p, nw, cmax, ct.byref(sc), ct.byref(lim)) == 0
    scale, limit = sc.value, lim.value
    S = math.log2(scale)
    assert S == int(S) and S <= 44
    deg = 2 * (p - 1) + 2 + 2 * nw + 1       # collision, energy, wall and fixed edges of a node
    assert deg * limit * scale <= 2.0 ** 62 * (1 + 1e-12)
    assert limit >= 8 * cmax


def test_consensus_scale_rejects_bad_arguments(lib):
    sc, lim = ct.c_double(), ct.c_double()
    for args in ((0, 0, 1.0), (4, -1, 1.0), (4, 0, 0.5), (4, 0, float("nan"))):
        assert lib.twa_consensus_scale(*args, ct.byref(sc), ct.byref(lim)) == 1


def test_set_allocator_takes_both_callbacks_or_none(lib):
    fn_a = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_int, ct.c_void_p, ct.c_void_p)
    fn_f = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_size_t, ct.c_int, ct.c_void_p, ct.c_void_p)
    lib.twa_set_allocator.restype = ct.c_int
    lib.twa_set_allocator.argtypes = [fn_a, fn_f, ct.c_void_p]
    a = fn_a(lambda n, d, s, c: None)
    f = fn_f(lambda p, n, d, s, c: None)
    assert lib.twa_set_allocator(a, fn_f(), None) == 1
    assert lib.twa_set_allocator(fn_a(), f, None) == 1
    assert lib.twa_set_allocator(a, f, None) == 0
    assert lib.twa_set_allocator(fn_a(), fn_f(), None) == 0
