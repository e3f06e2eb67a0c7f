"""Failure detection through the C ABI: infeasible or invalid problems at
create, non-finite and diverging states after iterating, calls in the wrong
state.  Every condition is forced from the host; every kernel exits
normally (the values involved are finite or are scanned, never indexed)."""
import numpy as np
import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu


def _twa():
    import paper_1311_4527_amd.twa as T
    return T


def _status_of_create(inst, flags=0, **over):
    T = _twa()
    args = dict(radii=inst.radii, x0=inst.x0, xT=inst.xT, walls=inst.walls if inst.n_walls else None, C=inst.C,
                rho0=inst.rho0, alpha=inst.alpha)
    args.update(over)
    try:
        S = T.Solver(inst.p, inst.eta, inst.dim, flags=flags, **args)
    except T.TWAError as e:
        return e.status
    S.close()
    return T.TWA_OK


def test_overlapping_starts_and_goals_are_infeasible():
    T = _twa()
    inst = I.random_box(5, 0.05, 3, seed=1, C=0.1)
    x0 = inst.x0.copy()
    x0[3] = x0[1] + np.array([0.06, 0.0])          # 0.06 apart, r_i + r_j = 0.1
    assert _status_of_create(inst, x0=x0) == T.TWA_E_INFEASIBLE
    xT = inst.xT.copy()
    xT[0] = xT[4] + np.array([0.0, -0.099])
    assert _status_of_create(inst, xT=xT) == T.TWA_E_INFEASIBLE
    # exactly in contact is feasible (non-strict separation, Sec. 3.1)
    x0 = inst.x0.copy()
    x0[3] = x0[1] + np.array([0.1, 0.0])
    if np.min(np.linalg.norm(x0[:, None] - x0[None], axis=2) + np.eye(5) * 9) >= 0.1 - 1e-7:
        assert _status_of_create(inst, x0=x0) == T.TWA_OK


def test_start_or_goal_within_radius_of_a_wall_is_infeasible():
    T = _twa()
    inst = I.random_box(4, 0.05, 3, n_walls=1, seed=2, C=0.1)
    walls = inst.walls.copy()
    a = inst.x0[2]
    walls[0] = [a + [0.03, -0.1], a + [0.03, 0.1]]  # vertical wall 0.03 from start 2
    assert _status_of_create(inst, walls=walls) == T.TWA_E_INFEASIBLE
    g = inst.xT[1]
    walls[0] = [g + [-0.1, 0.049], g + [0.1, 0.049]]
    assert _status_of_create(inst, walls=walls) == T.TWA_E_INFEASIBLE


def test_invalid_inputs():
    T = _twa()
    inst = I.random_box(4, 0.05, 3, n_walls=1, seed=3, C=0.1)
    x0 = inst.x0.copy()
    x0[1, 0] = np.nan
    assert _status_of_create(inst, x0=x0) == T.TWA_E_INVALID
    C = inst.C.copy()
    C[0, 0] = np.inf
    assert _status_of_create(inst, C=C) == T.TWA_E_INVALID
    r = inst.radii.copy()
    r[2] = 0.0
    assert _status_of_create(inst, radii=r) == T.TWA_E_INVALID
    assert _status_of_create(inst, rho0=0.0) == T.TWA_E_INVALID
    assert _status_of_create(inst, alpha=-1.0) == T.TWA_E_INVALID
    assert _status_of_create(inst, flags=T.TWA_F_COST_NONE | T.TWA_F_COST_MAXVEL) == T.TWA_E_INVALID
    assert _status_of_create(inst, flags=T.TWA_F_VO) == T.TWA_E_INVALID     # needs eta == 1
    assert _status_of_create(inst, flags=1 << 12) == T.TWA_E_INVALID
    assert _status_of_create(inst, flags=T.TWA_F_COST_MAXVEL, C=np.zeros_like(inst.C)) == T.TWA_E_INVALID


def test_non_finite_state_is_reported():
    import torch
    T = _twa()
    inst = I.random_box(6, 0.05, 4, seed=4, sigma=1e-2, alpha=0.1, C=1 / 24)
    S = T.Solver.from_instance(inst)
    S.twa_iterate(5)
    S.twa_check_finite()
    z, u, l, k = S.twa_get_state()
    u2 = u.clone()
    u2[u2.shape[0] // 2, 0] = float("nan")
    S.twa_set_state(z, u2, l, k)
    with pytest.raises(T.TWAError) as e:
        S.twa_check_finite()
    assert e.value.status == T.TWA_E_NUMERIC
    # a clean state clears it
    S.twa_set_state(z, u, l, k)
    S.twa_check_finite()


def test_consensus_overflow_is_reported():
    """A break-point far outside the scene (1e6, still finite in FP32) makes
    the consensus contributions of its node exceed the fixed-point headroom:
    the overflow flag turns into TWA_E_NUMERIC instead of a silently wrapped
    sum."""
    import torch
    T = _twa()
    inst = I.random_box(4, 0.05, 3, seed=5, sigma=1e-2, alpha=0.1, C=1 / 12)
    scale, limit = T.twa_consensus_scale(4, 0, 1.0)
    assert limit < 1e6
    S = T.Solver.from_instance(inst)
    z, u, l, k = S.twa_get_state()
    z2 = z.clone()
    z2[1, 1] = torch.tensor([1e6, -1e6])
    S.twa_set_state(z2, u, l, 0)
    S.twa_iterate(1)
    with pytest.raises(T.TWAError) as e:
        S.twa_check_finite()
    assert e.value.status == T.TWA_E_NUMERIC
    with pytest.raises(T.TWAError) as e:
        S.twa_get_stats()
    assert e.value.status == T.TWA_E_NUMERIC
    S.twa_set_state(z, u, l, 0)
    S.twa_iterate(3)
    S.twa_check_finite()
    assert S.twa_get_stats()["iter"] == 3


def test_backward_needs_tape_and_plane():
    T = _twa()
    inst = I.random_box(4, 0.05, 3, seed=6, sigma=1e-2, alpha=0.1, C=1 / 12)
    S = T.Solver.from_instance(inst)
    S.twa_iterate(2)
    with pytest.raises(T.TWAError) as e:
        S.twa_backward(np.zeros(inst.z0.shape))
    assert e.value.status == T.TWA_E_STATE
    inst3 = I.random_box(4, 0.05, 3, dim=3, seed=6, sigma=1e-2, alpha=0.1, C=1 / 12)
    S3 = T.Solver.from_instance(inst3, flags=T.TWA_F_TAPE)
    S3.twa_iterate(2)
    with pytest.raises(T.TWAError) as e:
        S3.twa_backward(np.zeros(inst3.z0.shape))
    assert e.value.status == T.TWA_E_INVALID


def test_stats_residual_and_measures():
    """twa_get_stats: the residual max |x - z| over the edges whose u the
    last iteration updated shrinks as a collision-free instance converges to
    its straight line, and the objective and clearance equal
    twa_get_quality's.  Reading the stats leaves the run bitwise unchanged."""
    import torch
    T = _twa()
    inst = I.random_box(6, 0.02, 4, seed=7, sigma=3e-2, alpha=0.1, C=1 / 24)
    S = T.Solver.from_instance(inst)
    R = T.Solver.from_instance(inst)
    assert S.twa_get_stats()["residual"] == 0.0
    S.twa_iterate(5)
    R.twa_iterate(5)
    st = S.twa_get_stats()
    r5 = st["residual"]
    q = S.twa_get_quality()
    assert r5 > 0 and st["objective"] == q["objective"] and st["min_clearance"] == q["min_clearance"]
    S.twa_iterate(400)
    R.twa_iterate(400)
    r405 = S.twa_get_stats()["residual"]
    assert r405 < 0.1 * r5
    assert torch.equal(S.twa_get_trajectories(), R.twa_get_trajectories())
