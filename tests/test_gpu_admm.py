"""Standard-ADMM mode (TWA_F_ADMM: every weight rho0) of the HIP planner
against the FP64 reference run in the same mode, whose all-rho0 iteration is
pinned to textbook consensus ADMM in the CPU suite."""
import numpy as np
import pytest

import oracle as O
from paper_1311_4527_amd import instances as I
from tests.test_gpu_parity import _reference_states, one_iteration_parity

pytestmark = pytest.mark.gpu


def _flags():
    from paper_1311_4527_amd.twa import TWA_F_ADMM
    return TWA_F_ADMM


@pytest.mark.parametrize("seed", [0, 1])
def test_admm_one_iteration_parity_swap(seed):
    inst = I.conf_small(seed)
    for k, z, u, lr in _reference_states(inst, [0, 1, 10, 100, 400], mode=O.MODE_ADMM):
        one_iteration_parity(inst, z, u, lr, k, flags=_flags(), mode=O.MODE_ADMM)


def test_admm_one_iteration_parity_walls():
    inst = I.random_box(20, 0.03, 5, n_walls=6, sigma=1e-2, seed=11, alpha=0.1, C=1 / 100)
    for k, z, u, lr in _reference_states(inst, [0, 3, 30, 150], mode=O.MODE_ADMM):
        one_iteration_parity(inst, z, u, lr, k, flags=_flags(), mode=O.MODE_ADMM)


def test_admm_end_points_are_not_pinned():
    """Under ADMM the start/goal factors take part in the consensus with
    weight rho0, so <-rho is rho0 at every node."""
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_small(0)
    S = Solver.from_instance(inst, flags=_flags())
    S.twa_iterate(5)
    z, u, lr, _ = S.twa_get_state()
    assert np.all(lr.cpu().numpy() == O.STD)


def test_admm_full_run_matches_reference():
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_small(0)
    S = Solver.from_instance(inst, flags=_flags())
    S.twa_iterate(3000)
    zg = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    P = O.Planner(inst, mode=O.MODE_ADMM)
    P.iterate(3000)
    Jg = float(np.sum(inst.C * np.sum(np.diff(zg, axis=1) ** 2, axis=2)))
    Jr = P.objective()
    assert abs(Jg - Jr) <= 1e-3 * Jr, (Jg, Jr)
    assert O.min_clearance(inst.radii, zg) > min(P.min_clearance(), 0.0) - 5e-5


@pytest.mark.parametrize("block", [256, 0])
def test_admm_batch_equals_plain(block):
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = I.conf_batch(6, base_seed=31, p_range=(4, 24))
    B = Batch(insts, flags=_flags())
    B.twa_batch_config(block, len(insts))
    B.twa_batch_iterate(30)
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst, flags=_flags())
        S.twa_iterate(30)
        assert torch.equal(B.twa_batch_get_trajectories(i), S.twa_get_trajectories())


def test_admm_one_iteration_parity_many_chunks():
    """150 agents with walls: rows of the pair triangle span up to three
    64-pair chunks plus a ragged tail, in ADMM's dense layout."""
    inst = I.random_box(150, 0.01, 6, n_walls=8, sigma=1e-2, seed=12, alpha=0.1, C=1 / 900)
    for k, z, u, lr in _reference_states(inst, [0, 4, 40], mode=O.MODE_ADMM):
        one_iteration_parity(inst, z, u, lr, k, flags=_flags(), mode=O.MODE_ADMM)
