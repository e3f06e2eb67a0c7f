"""The fixed start and goal factors (weight infinity, App. B step 5) decide
z at their nodes alone: after any iteration those break-points are exactly
the given start and goal, whatever the state the iteration started from
(which is also why no other factor's contribution to such a node is made)."""
import numpy as np
import pytest

from paper_1311_4527_amd import instances as I

pytestmark = pytest.mark.gpu

F_DENSE = 1
CASES = {
    "swap8": lambda: I.conf_small(0),                                       # one-workgroup path
    "box48_walls": lambda: I.conf_box1024(seed=9, p=48, eta=6, n_walls=4),  # plain kernels
}


def _ends(S, inst):
    z = S.twa_get_trajectories().cpu().numpy()
    assert np.array_equal(z[:, 0], inst.x0.astype(np.float32))
    assert np.array_equal(z[:, -1], inst.xT.astype(np.float32))


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("flags", [0, F_DENSE])
def test_fixed_ends_stay_exact(case, flags):
    from paper_1311_4527_amd.twa import Solver
    inst = CASES[case]()
    S = Solver.from_instance(inst, flags=flags)
    for k in (1, 37, 300):
        S.twa_iterate(k)
        _ends(S, inst)
    S.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_fixed_ends_restored_from_any_state(case):
    """A state whose end break-points are moved and marked as ordinary
    (weight rho0) nodes: one iteration puts them back exactly."""
    from paper_1311_4527_amd.twa import Solver
    inst = CASES[case]()
    rng = np.random.default_rng(4)
    S = Solver.from_instance(inst)
    S.twa_iterate(20)
    z, u, lr, it = S.twa_get_state()
    z = z.cpu().numpy().copy()
    lr = lr.cpu().numpy().copy()
    z[:, 0] += rng.normal(scale=0.01, size=z[:, 0].shape).astype(np.float32)
    z[:, -1] += rng.normal(scale=0.01, size=z[:, -1].shape).astype(np.float32)
    lr[:, 0] = 1
    lr[:, -1] = 1
    S.twa_set_state(z, u, lr, int(it))
    S.twa_iterate(1)
    _ends(S, inst)
    S.close()
