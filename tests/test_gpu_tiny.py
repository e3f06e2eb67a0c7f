"""Instances of at most 256 collision + wall factors (or 512 collision
factors and no walls): untimed iterations run in one workgroup, all
iterations of a call in one launch, with the whole state held in LDS when it
fits (else in the persistent batched kernel).
The per-factor code is the plain kernels', so the state after any mix of
such calls and plain iterations must equal, bit for bit, the state after
plain iterations alone (twa_iterate_timed launches its last two iterations
on their own, through the plain kernels, so calls of two timed iterations
run plain throughout)."""
import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu

F_DENSE, F_ADMM, F_NONE, F_MAXVEL, F_MINVEL = 1, 4, 8, 16, 32

CASES = {
    "swap8_2d": lambda: I.conf_small(0),                                # 112 collision factors
    "swap6_3d": lambda: I.circle_swap(6, 0.05, 4, dim=3, seed=3),       # 60
    "box8_walls": lambda: I.conf_box1024(seed=5, p=8, eta=4, n_walls=4),  # 112 + 128 wall factors
    # 190 collision factors over 191 break-points: 54 KiB of state in LDS, near
    # the bound; 250 over 251: too large for the LDS copy
    "pair_eta190": lambda: I.circle_swap(2, 0.05, 190, seed=4),
    "pair_eta250": lambda: I.circle_swap(2, 0.05, 250, seed=4),
    # more than 256 collision factors and no walls: owners on all eight waves
    "swap16_eta4": lambda: I.circle_swap(16, 0.05, 4, seed=6),          # 480
}


def _tiny(c):
    return c["coll"] + c["wall"] <= 256 or (c["wall"] == 0 and c["coll"] <= 512)


def _state(S):
    import torch
    z, u, lr, it = S.twa_get_state()
    torch.cuda.synchronize()
    return z.cpu(), u.cpu(), lr.cpu(), it


def _plain(S, k):
    assert k % 2 == 0
    for _ in range(k // 2):
        S.twa_iterate_timed(2)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("flags", [0, F_DENSE, F_ADMM, F_NONE, F_MAXVEL, F_MINVEL])
def test_tiny_equals_plain(case, flags):
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = CASES[case]()
    c = inst.counts()
    assert _tiny(c)
    A = Solver.from_instance(inst, flags=flags)
    B = Solver.from_instance(inst, flags=flags)
    A.twa_iterate(37)            # from the initial state
    A.twa_iterate_timed(3)       # plain iterations in between
    A.twa_iterate(260)           # a pending state carried into the kernel
    _plain(B, 300)
    za, ua, la, ia = _state(A)
    zb, ub, lb, ib = _state(B)
    assert ia == ib == 300
    assert torch.equal(za, zb)
    assert torch.equal(ua, ub)
    assert torch.equal(la, lb)
    sa, sb = A.twa_get_stats(), B.twa_get_stats()
    assert sa == sb
    A.close()
    B.close()


def test_tiny_after_warm_up_schedule():
    """Warm-up iterations (rho0_init) run plain; later calls take the kernel
    at rho0, the first of them with a previous iteration at rho0 too."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_small(1)
    A = Solver.from_instance(inst)
    B = Solver.from_instance(inst)
    for S in (A, B):
        S.twa_set_schedule(0.25, 12)
    A.twa_iterate(12)   # the warm-up
    A.twa_iterate(1)    # previous iteration in the warm-up: plain
    A.twa_iterate(199)
    _plain(B, 212)
    za, ua, la, _ = _state(A)
    zb, ub, lb, _ = _state(B)
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    A.close()
    B.close()


def test_tiny_long_call_spans_launches():
    """More iterations than one launch of the kernel runs (4096)."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_small(2)
    A = Solver.from_instance(inst)
    B = Solver.from_instance(inst)
    A.twa_iterate(5000)
    for _ in range(5):
        B.twa_iterate(1000)
    za, ua, la, ia = _state(A)
    zb, ub, lb, ib = _state(B)
    assert ia == ib == 5000
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    A.close()
    B.close()


@pytest.mark.parametrize("p", [12, 32])
def test_tiny_vo_epoch_equals_plain(p):
    """A velocity-obstacle epoch (eta = 1) in the LDS-resident kernel (32
    agents: 496 collision factors, owners on all eight waves)."""
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_VO
    inst = I.circle_swap(p, 0.05 if p == 12 else 0.03, 1, seed=5, alpha=0.1, C=0.05)
    A = Solver.from_instance(inst, flags=TWA_F_VO)
    B = Solver.from_instance(inst, flags=TWA_F_VO)
    A.twa_iterate(149)
    A.twa_iterate(1)
    _plain(B, 150)
    za, ua, la, _ = _state(A)
    zb, ub, lb, _ = _state(B)
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    A.close()
    B.close()


def _until_by_blocks(S, max_iter, every, bar):
    """The stopping rule of twa_iterate_until, from the host."""
    done = 0
    while done < max_iter:
        n = min(every, max_iter - done)
        S.twa_iterate(n)
        done += n
        if S.twa_get_quality()["min_clearance"] >= bar:
            return done, True
    return done, False


def _vo12():
    return I.circle_swap(12, 0.05, 1, seed=5, alpha=0.1, C=0.05)


UNTIL = [
    # (instance, flags, every, max_iter, bar): a VO epoch (stops partway), the
    # bar met at the first check, never met, a call longer than one launch
    # (4096 iterations) with a short last block, walls, an instance whose state
    # does not fit in LDS (host-driven blocks) and one too large for the
    # one-workgroup path
    ("vo12", "vo", 50, 20000, -5e-7),
    ("swap8_2d", 0, 30, 700, -float("inf")),
    ("swap8_2d", 0, 30, 700, float("inf")),
    ("swap8_2d", 0, 50, 5010, float("inf")),
    ("swap8_2d", 0, 1000, 40000, float("inf")),  # more than one group of 8 launches
    ("box8_walls", 0, 25, 1000, -1e-6),
    ("swap6_3d", 0, 30, 900, -1e-6),
    ("swap8_2d", 1, 40, 2000, -1e-6),  # dense form
    ("pair_eta250", 0, 40, 300, -1e-6),
    ("box16", 0, 20, 200, -1e-6),
    ("swap16_eta4", 0, 25, 600, -1e-6),
]


@pytest.mark.parametrize("case,flags,every,max_iter,bar", UNTIL)
def test_iterate_until_equals_host_blocks(case, flags, every, max_iter, bar):
    import torch
    from paper_1311_4527_amd.twa import Solver, TWA_F_VO
    make = {"vo12": _vo12, "box16": lambda: I.conf_box1024(seed=6, p=16, eta=4, n_walls=4), **CASES}[case]
    fl = TWA_F_VO if flags == "vo" else flags
    inst = make()
    A = Solver.from_instance(inst, flags=fl)
    B = Solver.from_instance(inst, flags=fl)
    A.twa_iterate(7)  # a pending state carried into the call
    B.twa_iterate(7)
    got = A.twa_iterate_until(max_iter, every, bar)
    want = _until_by_blocks(B, max_iter, every, bar)
    print(case, got, want, flush=True)
    assert got == want
    za, ua, la, ia = _state(A)
    zb, ub, lb, ib = _state(B)
    assert ia == ib == 7 + got[0]
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    assert A.twa_get_stats() == B.twa_get_stats()
    A.close()
    B.close()


def test_iterate_until_rejects_bad_arguments():
    from paper_1311_4527_amd.twa import Solver, TWAError
    S = Solver.from_instance(I.conf_small(0))
    for args in [(-1, 10, 0.0), (10, 0, 0.0), (10, 5, float("nan"))]:
        with pytest.raises(TWAError):
            S.twa_iterate_until(*args)
    assert S.twa_iterate_until(0, 5, 0.0) == (0, False)
    S.close()


def test_iterate_until_through_a_warm_up_schedule():
    """Blocks that start inside a rho0 warm-up run from the host (plain
    iterations at the warm-up value); the result equals the host loop."""
    import torch
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_small(1)
    A = Solver.from_instance(inst)
    B = Solver.from_instance(inst)
    for S in (A, B):
        S.twa_set_schedule(0.25, 30)
    got = A.twa_iterate_until(400, 25, -1e-6)
    want = _until_by_blocks(B, 400, 25, -1e-6)
    assert got == want
    za, ua, la, ia = _state(A)
    zb, ub, lb, ib = _state(B)
    assert ia == ib
    assert torch.equal(za, zb) and torch.equal(ua, ub) and torch.equal(la, lb)
    A.close()
    B.close()
