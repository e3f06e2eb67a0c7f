"""Batched instances (one persistent launch, or one launch per phase over
all instances) evolve bitwise as the same instances do in their own
solvers; ragged p, eta, 2-D and 3-D, walls."""
import numpy as np
import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu


def _mixed(n=12, seed=5):
    out = I.conf_batch(n, base_seed=seed, p_range=(4, 40))
    return out


@pytest.mark.parametrize("block,groups", [(256, 12), (512, 3), (1024, 1), (256, 5), (0, 1)])
def test_batch_equals_plain(block, groups):
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = _mixed()
    B = Batch(insts)
    B.twa_batch_config(block, groups)
    B.twa_batch_iterate(40)
    B.twa_batch_iterate(25)
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst)
        S.twa_iterate(65)
        a = B.twa_batch_get_trajectories(i)
        b = S.twa_get_trajectories()
        assert torch.equal(a, b), (i, inst.name, (a - b).abs().max().item())
        za, ua, la, ka = B.twa_batch_solver(i).twa_get_state()
        zb, ub, lb, kb = S.twa_get_state()
        assert ka == kb == 65 and torch.equal(ua, ub) and torch.equal(la, lb)


@pytest.mark.parametrize("block,groups,flags", [(1024, 2, 0), (512, 5, 1), (0, 1, 0), (0, 1, 1)])
def test_batch_equals_plain_long_rows(block, groups, flags):
    """Instances with p >= 64 take the column walk in the persistent kernel."""
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = I.conf_batch(6, base_seed=21, p_range=(60, 100))
    B = Batch(insts, flags=flags)
    B.twa_batch_config(block, groups)
    B.twa_batch_iterate(30)
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst, flags=flags)
        S.twa_iterate(30)
        a, b = B.twa_batch_get_trajectories(i), S.twa_get_trajectories()
        assert torch.equal(a, b), (i, inst.name, (a - b).abs().max().item())


def test_batch_dense_equals_skip():
    import torch
    from paper_1311_4527_amd.twa import Batch, TWA_F_DENSE
    insts = _mixed(8, seed=9)
    A = Batch(insts, flags=0)
    D = Batch(insts, flags=TWA_F_DENSE)
    A.twa_batch_iterate(30)
    D.twa_batch_iterate(30)
    for i in range(len(insts)):
        assert torch.equal(A.twa_batch_get_trajectories(i), D.twa_batch_get_trajectories(i))


def test_batch_against_reference_one_iteration():
    """Instance by instance, one batched iteration equals the FP64 reference
    to the single-iteration tolerance."""
    import oracle as O
    from paper_1311_4527_amd.twa import Batch
    insts = _mixed(6, seed=13)
    B = Batch(insts)
    B.twa_batch_iterate(1)
    for i, inst in enumerate(insts):
        P = O.Planner(inst)
        z32 = inst.z0.astype(np.float32).astype(np.float64)
        P.set_state(z32, np.zeros((P.E, inst.dim)), P.get_state()[2], 0)
        P.iterate(1)
        zr = P.trajectories()
        zg = B.twa_batch_get_trajectories(i).cpu().numpy()
        act, tie = P.margins()
        if ((act < 1e-5) | (tie < 1e-5)).any():
            continue
        assert np.all(np.abs(zg - zr) <= 1e-5 * np.maximum(np.abs(zr), 1.0)), inst.name


def test_autotuner_picks_a_candidate(tmp_path, monkeypatch):
    monkeypatch.setenv("TWA_TUNE_CACHE", str(tmp_path / "tune.json"))
    import importlib
    import paper_1311_4527_amd.autotune as AT
    importlib.reload(AT)
    from paper_1311_4527_amd.twa import Batch
    B = Batch(_mixed(10, seed=3))
    log = []
    b, g = AT.tune(B, iters=3, log=log)
    assert (b, g) in AT.candidates(10) and len(log) == len(AT.candidates(10))
    assert AT.tune(B, iters=3) == (b, g)   # cached


@pytest.mark.parametrize("block,groups,flags", [(256, 3, 0), (1024, 1, 1), (0, 1, 0), (0, 1, 1)])
def test_batch_with_degenerate_members(block, groups, flags):
    """Members with no collision factor (one agent), one interval (eta = 1),
    two agents, a 3-D triple and a long-row box with walls, in one batch:
    each evolves bitwise as in its own solver."""
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = [I.conf_box1024(seed=3, p=1, eta=1, n_walls=2), I.circle_swap(1, 0.05, 5, seed=1),
             I.circle_swap(2, 0.05, 1, seed=2), I.circle_swap(3, 0.05, 2, dim=3, seed=3),
             I.conf_box1024(seed=4, p=70, eta=4, n_walls=3), I.conf_small(0)]
    B = Batch(insts, flags=flags)
    B.twa_batch_config(block, groups)
    B.twa_batch_iterate(30)
    B.twa_batch_iterate(7)
    for i, inst in enumerate(insts):
        S = Solver.from_instance(inst, flags=flags)
        S.twa_iterate(37)
        a, b = B.twa_batch_get_trajectories(i), S.twa_get_trajectories()
        assert torch.equal(a, b), (i, inst.name, (a - b).abs().max().item())
        za, ua, la, ka = B.twa_batch_solver(i).twa_get_state()
        zb, ub, lb, kb = S.twa_get_state()
        assert ka == kb == 37 and torch.equal(ua, ub) and torch.equal(la, lb)
        S.close()
    B.close()
