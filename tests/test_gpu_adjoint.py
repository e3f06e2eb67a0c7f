"""The HIP adjoint of unrolled iterations (twa_backward, through the C ABI)
against the FP64 reference adjoint, which is itself pinned to FP64 central
differences of the unrolled map.

Both sides receive the same seeded cotangent dL/dz^K (a linear loss), so the
comparison is of J^T v for one v.  Bar, element by element: |gpu - ref| <=
1e-3 * max(|ref|, 0.1 * max|ref of that output|).  The floor: an entry far
below its output's largest is a sum in which larger FP32 terms cancel, so its
rounding error scales with the output's magnitude, not its own."""
import numpy as np
import pytest

import oracle as O
from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu

REL = 1e-3
FLOOR = 0.1


def _sub(seed=7, radius=None):
    inst = I.sub_instance(I.conf_adjoint(seed), np.arange(0, 256, 32))
    if radius is not None:
        inst.radii[:] = radius
    return inst


def _gpu_grad(inst, K, v):
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    S.twa_iterate(K)
    out = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(torch.from_numpy(v.astype(np.float32)))]
    z = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    S.close()
    return out, z


def _ref_grad(inst, K, v):
    P = O.Planner(inst)
    P.tape(K)
    return P.backward(v), P.trajectories()


def _compare(got, ref, names=("dx0", "dxT", "dr", "dz0")):
    for name, a, b in zip(names, got, ref):
        scale = max(np.abs(b).max(), 1e-12)
        tol = REL * np.maximum(np.abs(b), FLOOR * scale)
        err = np.abs(a - b)
        worst = float(np.max(err / tol))
        print(f"{name}: max|ref| {scale:.3e}  max err {err.max():.3e}  worst err/tol {worst:.2f}", flush=True)
        assert np.all(err <= tol), (name, np.argwhere(err > tol)[:5].ravel(), worst)


@pytest.mark.parametrize("K", [1, 6, 40])
def test_adjoint_matches_reference_colliding(K):
    """p=8 swap with large radii: many collision factors active."""
    inst = _sub(radius=0.3)
    v = np.random.default_rng(100 + K).normal(size=inst.z0.shape)
    (g_gpu, z_gpu), (g_ref, z_ref) = _gpu_grad(inst, K, v), _ref_grad(inst, K, v)
    assert np.abs(z_gpu - z_ref).max() < 1e-4
    _compare(g_gpu, g_ref)
    assert np.abs(g_ref[2]).max() > 0  # the radii matter


def test_adjoint_matches_reference_K500():
    """The differentiable workload's p=8 sub-instance (agents 0, 32, ..., 224
    of the p=256 swap, r=0.008, eta=8) over K=500 iterations (sqrt(K)
    checkpointing: segments of 23)."""
    inst = _sub()
    v = np.random.default_rng(5).normal(size=inst.z0.shape)
    (g_gpu, z_gpu), (g_ref, z_ref) = _gpu_grad(inst, 500, v), _ref_grad(inst, 500, v)
    _compare(g_gpu, g_ref)


def test_adjoint_with_walls():
    inst = I.random_box(6, 0.08, 4, n_walls=3, sigma=1e-2, seed=4, alpha=0.1, C=1 / 24)
    v = np.random.default_rng(9).normal(size=inst.z0.shape)
    for K in (5, 30):
        (g_gpu, _), (g_ref, _) = _gpu_grad(inst, K, v), _ref_grad(inst, K, v)
        _compare(g_gpu, g_ref)


def test_backward_leaves_forward_state():
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = _sub(radius=0.2)
    A = Solver.from_instance(inst, flags=TWA_F_TAPE)
    B = Solver.from_instance(inst)
    A.twa_iterate(37)
    B.twa_iterate(37)
    A.twa_backward(torch.ones(inst.z0.shape))
    A.twa_iterate(20)
    B.twa_iterate(20)
    za, ua, la, ia = A.twa_get_state()
    zb, ub, lb, ib = B.twa_get_state()
    assert ia == ib == 57
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)


def test_backward_needs_tape_flag():
    import torch
    from paper_1311_4527_amd.twa import Solver, TWAError, TWA_E_STATE
    inst = _sub()
    S = Solver.from_instance(inst)
    S.twa_iterate(2)
    with pytest.raises(TWAError) as e:
        S.twa_backward(torch.ones(inst.z0.shape))
    assert e.value.status == TWA_E_STATE


def test_zero_iterations_is_identity_on_the_init():
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = _sub()
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    v = torch.arange(inst.z0.size, dtype=torch.float32).reshape(inst.z0.shape)
    dx0, dxT, dr, dz0 = S.twa_backward(v)
    vn = v.numpy()
    assert np.array_equal(dx0.cpu().numpy(), vn[:, 0])
    assert np.array_equal(dxT.cpu().numpy(), vn[:, -1])
    assert np.all(dr.cpu().numpy() == 0)
    exp = vn.copy()
    exp[:, 0] = 0
    exp[:, -1] = 0
    assert np.array_equal(dz0.cpu().numpy(), exp)


def test_autograd_function_chains_through_the_straight_line_init():
    """TWASolve behind torch.autograd: with z0 built from x0 and xT in torch,
    dL/dx0 = the adjoint's dx0 plus the interior dz0 carried back through the
    straight line."""
    import torch
    from paper_1311_4527_amd.autograd import solve
    inst = _sub(radius=0.3)
    dev = "cuda"
    x0 = torch.tensor(inst.x0, dtype=torch.float32, device=dev, requires_grad=True)
    xT = torch.tensor(inst.xT, dtype=torch.float32, device=dev, requires_grad=True)
    r = torch.tensor(inst.radii, dtype=torch.float32, device=dev, requires_grad=True)
    C = torch.tensor(inst.C, dtype=torch.float32, device=dev)
    z = solve(x0, xT, r, 12, inst.eta, C=C, rho0=inst.rho0, alpha=inst.alpha)
    target = torch.zeros_like(z)
    loss = (C * ((z[:, 1:] - z[:, :-1]) ** 2).sum(-1)).sum() + 0.5 * ((z - target) ** 2).sum()
    loss.backward()
    # the reference: the same loss through the FP64 adjoint, the straight-line
    # init chained by hand
    ref = I.sub_instance(I.conf_adjoint(7), np.arange(0, 256, 32))
    ref.radii[:] = 0.3
    t = np.linspace(0, 1, inst.eta + 1)[None, :, None]
    ref.z0 = ref.x0[:, None, :] + t * (ref.xT - ref.x0)[:, None, :]
    P = O.Planner(ref)
    P.tape(12)
    zr = P.trajectories()
    d = np.diff(zr, axis=1)
    w = 2 * ref.C[..., None] * d
    v = np.zeros_like(zr)
    v[:, 1:] += w
    v[:, :-1] -= w
    v += zr
    dx0, dxT, dr, dz0 = P.backward(v)
    dx0 = dx0 + np.sum((1 - t) * dz0, axis=1)
    dxT = dxT + np.sum(t * dz0, axis=1)
    _compare([x0.grad.cpu().numpy(), xT.grad.cpu().numpy(), r.grad.cpu().numpy()], [dx0, dxT, dr],
             names=("dx0", "dxT", "dr"))


def test_full_size_adjoint_runs_and_is_linear():
    """p=256, eta=8, K=500 (1,049,088 edges): the adjoint runs with sqrt(K)
    checkpoints, is finite, and is linear in the cotangent."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = I.conf_adjoint(7)
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    S.twa_iterate(500)
    rng = np.random.default_rng(3)
    v1 = torch.from_numpy(rng.normal(size=inst.z0.shape).astype(np.float32))
    v2 = torch.from_numpy(rng.normal(size=inst.z0.shape).astype(np.float32))
    g1 = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(v1)]
    g2 = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(v2)]
    g12 = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(v1 + 2 * v2)]
    for a, b, c in zip(g1, g2, g12):
        assert np.all(np.isfinite(c))
        scale = max(np.abs(c).max(), 1e-12)
        assert np.abs(a + 2 * b - c).max() <= 1e-4 * scale
    S.close()


@pytest.mark.parametrize("case", ["swap100", "box64_walls", "swap8_tiny"])
@pytest.mark.parametrize("flags", [0, 1])
def test_reading_the_state_leaves_the_run_unchanged(case, flags):
    """The adjoint takes a checkpoint every ceil(sqrt(K)) iterations
    (twa_get_state settles the deferred u update, and the next iteration
    starts afresh) and recomputes each segment from it; the states it
    linearises about must be the forward run's own, bit for bit."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = {"swap100": lambda: I.conf_swap100(0),
            "box64_walls": lambda: I.conf_box1024(seed=9, p=64, eta=8, n_walls=4),
            "swap8_tiny": lambda: I.conf_small(0)}[case]()
    A = Solver.from_instance(inst, flags=flags)
    B = Solver.from_instance(inst, flags=flags)
    A.twa_iterate(100)
    for _ in range(100):
        B.twa_iterate(1)
        B.twa_get_state()
    za, ua, la, ia = A.twa_get_state()
    zb, ub, lb, ib = B.twa_get_state()
    torch.cuda.synchronize()
    assert ia == ib == 100
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    A.close()
    B.close()


def _tape_solver(inst, K, v):
    """A TAPE solver whose first backward made the forward tape, restarted
    from the initial state and run K iterations again (recorded)."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    S = Solver.from_instance(inst, flags=TWA_F_TAPE)
    S.twa_iterate(K)
    first = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(torch.from_numpy(v.astype(np.float32)))]
    S.twa_set_init(inst.z0)
    S.twa_iterate(K)
    return S, first


@pytest.mark.parametrize("K", [40, 500])
def test_forward_tape_matches_reference(K):
    """The second backward reads its checkpoints from the tape the forward
    recorded (no re-run of the forward): the same gradient as the reference
    and as the first call, the forward itself bitwise the untaped one, and
    the run continues bitwise afterwards."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = _sub(radius=0.3) if K == 40 else _sub()
    v = np.random.default_rng(11 + K).normal(size=inst.z0.shape)
    S, first = _tape_solver(inst, K, v)
    assert S.twa_get_stats()["tape_checkpoints"] == (K + 31) // 32
    R = Solver.from_instance(inst)
    R.twa_iterate(K)
    assert torch.equal(S.twa_get_trajectories(), R.twa_get_trajectories())
    got = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(torch.from_numpy(v.astype(np.float32)))]
    g_ref, _ = _ref_grad(inst, K, v)
    _compare(got, g_ref)
    for name, a, b in zip(("dx0", "dxT", "dr", "dz0"), got, first):
        scale = max(np.abs(b).max(), 1e-30)
        assert np.allclose(a, b, rtol=1e-4, atol=1e-4 * scale), (name, np.abs(a - b).max(), scale)
    assert torch.equal(S.twa_get_trajectories(), R.twa_get_trajectories())
    S.twa_iterate(9)
    R.twa_iterate(9)
    assert torch.equal(S.twa_get_trajectories(), R.twa_get_trajectories())
    S.close()
    R.close()


def test_forward_tape_outgrown_falls_back():
    """A run longer than the tape holds (64 checkpoints of 32 iterations) is
    differentiated by re-running the forward, with the same result as a
    solver that never had a tape."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = _sub()
    K = 2100
    v = np.random.default_rng(3).normal(size=inst.z0.shape)
    S, _ = _tape_solver(inst, 40, v)
    S.twa_set_init(inst.z0)
    S.twa_iterate(K)
    assert S.twa_get_stats()["tape_checkpoints"] == 0   # outgrown: no longer recording
    got = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(torch.from_numpy(v.astype(np.float32)))]
    F = Solver.from_instance(inst, flags=TWA_F_TAPE)
    F.twa_iterate(K)
    want = [t.cpu().numpy().astype(np.float64) for t in F.twa_backward(torch.from_numpy(v.astype(np.float32)))]
    for name, a, b in zip(("dx0", "dxT", "dr", "dz0"), got, want):
        assert np.all(np.isfinite(a)), name
        scale = max(np.abs(b).max(), 1e-30)
        assert np.allclose(a, b, rtol=1e-4, atol=1e-4 * scale), (name, np.abs(a - b).max(), scale)
    S.close()
    F.close()


def test_iterate_until_with_a_forward_tape():
    """twa_iterate_until on a solver that records a forward tape runs its
    blocks through the taped iteration (checkpoints every 32 iterations
    across blocks of 25), and the backward over that run equals the one of a
    plain run of the same length."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_TAPE
    inst = _sub(radius=0.3)
    v = np.random.default_rng(5).normal(size=inst.z0.shape)
    S, _ = _tape_solver(inst, 40, v)
    S.twa_set_init(inst.z0)
    done, met = S.twa_iterate_until(400, 25, float("inf"))  # a bar never met: all 16 blocks run
    assert (done, met) == (400, False)
    assert S.twa_get_stats()["tape_checkpoints"] == (done + 31) // 32
    F = Solver.from_instance(inst, flags=TWA_F_TAPE)
    F.twa_iterate(done)
    assert torch.equal(S.twa_get_trajectories(), F.twa_get_trajectories())
    vt = torch.from_numpy(v.astype(np.float32))
    got = [t.cpu().numpy().astype(np.float64) for t in S.twa_backward(vt)]
    want = [t.cpu().numpy().astype(np.float64) for t in F.twa_backward(vt)]
    for name, a, b in zip(("dx0", "dxT", "dr", "dz0"), got, want):
        scale = max(np.abs(b).max(), 1e-30)
        assert np.allclose(a, b, rtol=1e-4, atol=1e-4 * scale), (name, np.abs(a - b).max(), scale)
    S.close()
    F.close()
