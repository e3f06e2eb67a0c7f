"""twa_get_quality against the FP64 reference's clearance and the energy
objective's definition, on seeded synthetic break-points loaded with
twa_set_init (so no expected value comes from the GPU's own iterations):
the smallest clearance over every pair and interval and every wall, the
objective sum C |z_i(s+1) - z_i(s)|^2 (Sec. 2, 3.1, 3.2), and the largest move
of a break-point over the last iteration."""
import numpy as np
import pytest

import oracle as O
from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu


def _synthetic_z(inst, seed, sigma):
    """Straight lines from start to goal plus seeded noise, ends exact, FP32."""
    rng = np.random.default_rng(seed)
    s = np.linspace(0.0, 1.0, inst.eta + 1)[None, :, None]
    z = inst.x0[:, None, :] * (1 - s) + inst.xT[:, None, :] * s
    z = z + rng.normal(0.0, sigma, z.shape)
    z[:, 0] = inst.x0
    z[:, -1] = inst.xT
    return z.astype(np.float32)


def _expected(inst, z):
    z64 = z.astype(np.float64)
    radii = inst.radii.astype(np.float32).astype(np.float64)
    walls = inst.walls.reshape(-1, 4).astype(np.float32).astype(np.float64) if inst.n_walls else None
    clear = O.min_clearance(radii, z64, walls)
    C = inst.C.astype(np.float32).astype(np.float64)
    obj = float(np.sum(C * np.sum(np.diff(z64, axis=1) ** 2, axis=2)))
    return obj, clear


CASES = {
    "box32_walls": lambda: I.conf_box1024(seed=11, p=32, eta=8, n_walls=6),
    "swap12_3d": lambda: I.circle_swap(12, 0.05, 6, dim=3, seed=4),
    "single_agent_walls": lambda: I.conf_box1024(seed=3, p=1, eta=5, n_walls=4),
    "box1024_full": lambda: I.conf_box1024(),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_quality_matches_reference(case):
    from paper_1311_4527_amd.twa import Solver
    inst = CASES[case]()
    S = Solver.from_instance(inst)
    z = _synthetic_z(inst, 17, 0.05)
    S.twa_set_init(z)
    q = S.twa_get_quality()
    obj, clear = _expected(inst, z)
    assert q["max_move"] == 0.0
    assert abs(q["objective"] - obj) <= 1e-12 * max(obj, 1.0)
    if np.isinf(clear):
        assert np.isinf(q["min_clearance"]) and q["min_clearance"] > 0
    else:
        assert abs(q["min_clearance"] - clear) <= 1e-9
    S.close()


def test_quality_of_straight_line_swap_is_a_collision():
    """From create's straight lines every agent of a circle swap passes the
    centre at once: the clearance is -(r_i + r_j) up to the start noise."""
    from paper_1311_4527_amd.twa import Solver
    inst = I.circle_swap(8, 0.05, 4, sigma=0.0, seed=0)
    S = Solver.from_instance(inst, set_init=False)
    q = S.twa_get_quality()
    # create's straight lines: a + (s / eta)(b - a) in double from the FP32
    # start and goal, rounded to FP32
    a = inst.x0.astype(np.float32).astype(np.float64)[:, None, :]
    b = inst.xT.astype(np.float32).astype(np.float64)[:, None, :]
    z = (a + (np.arange(inst.eta + 1) / inst.eta)[None, :, None] * (b - a)).astype(np.float32)
    z[:, 0], z[:, -1] = a[:, 0], b[:, 0]
    obj, clear = _expected(inst, z)
    assert abs(q["min_clearance"] - clear) <= 1e-9
    assert q["min_clearance"] < -0.09
    assert abs(q["objective"] - obj) <= 1e-12 * max(obj, 1.0)
    S.close()


def test_max_move_is_the_last_iteration_step():
    from paper_1311_4527_amd.twa import Solver
    inst = I.conf_box1024(seed=11, p=32, eta=8, n_walls=6)
    S = Solver.from_instance(inst)
    S.twa_set_init(_synthetic_z(inst, 5, 0.05))
    S.twa_iterate(10)
    z0 = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    S.twa_iterate(1)
    z1 = S.twa_get_trajectories().cpu().numpy().astype(np.float64)
    q = S.twa_get_quality()
    want = float(np.max(np.sqrt(np.sum((z1 - z0) ** 2, axis=-1))))
    assert want > 0
    assert abs(q["max_move"] - want) <= 1e-12 * max(want, 1.0)
    S.close()
