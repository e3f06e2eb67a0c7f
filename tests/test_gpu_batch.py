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


@pytest.mark.parametrize("block,groups", [(0, 1), (256, 6)])
def test_batch_against_reference_one_iteration(block, groups):
    """Instance by instance, the first batched iteration equals the FP64
    reference by the single-iteration protocol: x per edge and ->rho per
    factor (captured through the batch), z, <-rho and u; near-tied factors
    validated and followed through, none skipped."""
    import torch
    import oracle as O
    from paper_1311_4527_amd.twa import Batch
    from tests.parity import compare_iteration
    insts = _mixed(6, seed=13)
    B = Batch(insts)
    B.twa_batch_config(block, groups)
    bufs = []
    for i, inst in enumerate(insts):
        S = B.twa_batch_solver(i)
        x = torch.empty((S.n_edges, inst.dim), dtype=torch.float32, device="cuda")
        r = torch.empty((S.n_factors,), dtype=torch.uint8, device="cuda")
        S.twa_capture_next(x, r)
        bufs.append((S, x, r))
    B.twa_batch_iterate(1)
    torch.cuda.synchronize()
    checked = []
    for inst, (S, x, r) in zip(insts, bufs):
        z, u, l, it = S.twa_get_state()
        assert it == 1
        lr0 = O.Planner(inst).get_state()[2]
        gpu = tuple(t.cpu().numpy() for t in (x, r, z, u, l))
        compare_iteration(inst, inst.z0.astype(np.float32), np.zeros((S.n_edges, inst.dim), np.float32), lr0, 0,
                          gpu)
        checked.append(inst.name)
    assert len(checked) == len(insts) and sum("swap" in n for n in checked) == 3, checked


def test_batch_after_warm_up_equals_plain():
    """A member that ran its warm-up schedule (Sec. 4's small rho0) through
    its own solver, with the last warm-up iteration's u update still pending,
    continues in the batch bitwise as in its own solver."""
    import torch
    from paper_1311_4527_amd.twa import Batch, Solver
    insts = _mixed(4, seed=17)
    B = Batch(insts)
    plain = []
    for i, inst in enumerate(insts):
        M = B.twa_batch_solver(i)
        M.twa_set_schedule(0.5, 3)
        M.twa_iterate(3)
        S = Solver.from_instance(inst)
        S.twa_set_schedule(0.5, 3)
        S.twa_iterate(3 + 20)
        plain.append(S)
    B.twa_batch_iterate(20)
    for i, S in enumerate(plain):
        za, ua, la, ka = B.twa_batch_solver(i).twa_get_state()
        zb, ub, lb, kb = S.twa_get_state()
        assert ka == kb == 23
        assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb), insts[i].name


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
