"""The other per-segment factors on the GPU: no cost (feasibility only,
Sec. 4), maximum and minimum velocity limits (eq. max_vel_min, App. F, G),
against the FP64 reference with the same factors."""
import numpy as np
import pytest

import oracle as O
from paper_1311_4527_amd import instances as I
from tests.test_gpu_parity import _reference_states, one_iteration_parity

pytestmark = pytest.mark.gpu


def _flag(cost):
    from paper_1311_4527_amd import twa
    return {O.COST_NONE: twa.TWA_F_COST_NONE, O.COST_MAXVEL: twa.TWA_F_COST_MAXVEL,
            O.COST_MINVEL: twa.TWA_F_COST_MINVEL}[cost]


def _limited(inst, factor):
    """Velocity limit per segment: factor x the straight-line step."""
    seg = np.linalg.norm(inst.xT - inst.x0, axis=1) / inst.eta
    inst.C = np.repeat((seg * factor)[:, None], inst.eta, axis=1)
    return inst


CASES = [(O.COST_NONE, None), (O.COST_MAXVEL, 1.3), (O.COST_MINVEL, 0.8)]


@pytest.mark.parametrize("cost,factor", CASES)
@pytest.mark.parametrize("dense", [0, 1])
def test_one_iteration_parity(cost, factor, dense):
    from paper_1311_4527_amd.twa import TWA_F_DENSE
    inst = I.conf_small(2)
    if factor is not None:
        _limited(inst, factor)
    flags = _flag(cost) | (TWA_F_DENSE if dense else 0)
    for k, z, u, lr in _reference_states(inst, [0, 1, 10, 100, 300], cost=cost):
        one_iteration_parity(inst, z, u, lr, k, flags=flags, cost=cost)


@pytest.mark.parametrize("cost,factor", CASES)
def test_one_iteration_parity_walls(cost, factor):
    inst = I.random_box(16, 0.03, 5, n_walls=5, sigma=1e-2, seed=8, alpha=0.1, C=1.0)
    if factor is not None:
        _limited(inst, factor)
    for k, z, u, lr in _reference_states(inst, [0, 5, 60], cost=cost):
        one_iteration_parity(inst, z, u, lr, k, flags=_flag(cost), cost=cost)


@pytest.mark.parametrize("cost,factor", [(O.COST_MAXVEL, 1.6), (O.COST_MINVEL, 0.7)])
def test_velocity_limits_hold_at_convergence(cost, factor):
    from paper_1311_4527_amd.twa import Solver
    inst = _limited(I.conf_small(1), factor)
    S = Solver.from_instance(inst, flags=_flag(cost))
    S.twa_iterate(3000)
    z = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    steps = np.linalg.norm(np.diff(z, axis=1), axis=2)
    if cost == O.COST_MINVEL:
        assert np.all(steps >= inst.C * (1 - 1e-3))
    else:
        assert np.all(steps <= inst.C * (1 + 1e-3))
    assert O.min_clearance(inst.radii, z) > -1e-4


def test_feasibility_restart_from_an_early_stop():
    """App. J: stopped early, the planner's state is a good start for the
    feasibility problem, which then finds a collision-free plan quickly."""
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_swap100(0)
    E = Solver.from_instance(inst)
    E.twa_iterate(200)
    z = E.twa_get_trajectories().cpu().numpy().astype(np.float64)
    assert O.min_clearance(inst.radii, z) < -1e-6  # not feasible yet
    F = Solver.from_instance(inst, flags=_flag(O.COST_NONE))
    zz, u, lr, it = E.twa_get_state()
    F.twa_set_state(zz, u, lr, 0)
    free = None
    for k in range(1, 41):
        F.twa_iterate(25)
        z = F.twa_get_trajectories().cpu().numpy().astype(np.float64)
        if O.min_clearance(inst.radii, z) >= -1e-6:
            free = 25 * k
            break
    assert free is not None


@pytest.mark.parametrize("block", [256, 0])
def test_batch_equals_plain_with_velocity_limits(block):
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = [_limited(i, 1.4) for i in I.conf_batch(6, base_seed=77, p_range=(4, 20))]
    B = Batch(insts, flags=_flag(O.COST_MAXVEL))
    B.twa_batch_config(block, len(insts))
    B.twa_batch_iterate(40)
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst, flags=_flag(O.COST_MAXVEL))
        S.twa_iterate(40)
        assert torch.equal(B.twa_batch_get_trajectories(i), S.twa_get_trajectories())


@pytest.mark.parametrize("cost,factor", CASES)
@pytest.mark.parametrize("dense", [0, 1])
def test_one_iteration_parity_many_chunks(cost, factor, dense):
    """140 agents with walls (multi-chunk rows and a ragged tail) for each
    per-segment factor, both layouts."""
    from paper_1311_4527_amd.twa import TWA_F_DENSE
    inst = I.random_box(140, 0.01, 5, n_walls=6, sigma=1e-2, seed=21, alpha=0.1, C=1.0)
    if factor is not None:
        _limited(inst, factor)
    flags = _flag(cost) | (TWA_F_DENSE if dense else 0)
    for k, z, u, lr in _reference_states(inst, [0, 6, 50], cost=cost):
        one_iteration_parity(inst, z, u, lr, k, flags=flags, cost=cost)
