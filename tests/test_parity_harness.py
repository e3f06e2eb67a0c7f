"""The single-iteration parity protocol (tests/parity.py) checked on the CPU
with the reference standing in for the GPU, and mistakes planted in its
outputs: the protocol must accept an equally good member of a tied argmin
followed through the consensus, and reject everything else (no GPU)."""
import numpy as np
import pytest

import oracle as O
from paper_1311_4527_amd import instances as I
from tests.parity import Layout, compare_iteration


def _head_on():
    """Two agents of radius 1/4 swapping along the x axis in two intervals,
    the middle break-points 0.2 apart on the axis: the instance is symmetric
    under y -> -y.  In the first interval the agents only need to move apart
    along the axis (a unique optimum); in the second they cross, and the
    sidestep up and its reflection down cost the same (an exact tie)."""
    x0 = np.array([[-1.0, 0.0], [1.0, 0.0]])
    xT = -x0
    z0 = np.array([[[-1.0, 0.0], [-0.1, 0.0], [1.0, 0.0]], [[1.0, 0.0], [0.1, 0.0], [-1.0, 0.0]]])
    return I.Instance(p=2, eta=2, dim=2, radii=np.full(2, 0.25), x0=x0, xT=xT, walls=np.zeros((0, 2, 2)),
                      C=np.full((2, 2), 0.25), z0=z0, rho0=1.0, alpha=0.1, name="head_on")


def _run(inst, override=None):
    P = O.Planner(inst)
    z, u, lr = P.get_state()
    if override is not None:
        P.override_next(*override)
    P.iterate(1)
    x, rf = P.last()
    zz, uu, ll = P.get_state()
    return (z.astype(np.float32), u.astype(np.float32), lr), [x, rf, zz, uu, ll]


def _mirrored(x, L, f):
    xm = x[L.edges(f)].copy()
    xm[:, 1] *= -1.0
    return xm


def test_identical_outputs_pass():
    inst = _head_on()
    (z, u, lr), gpu = _run(inst)
    info = compare_iteration(inst, z, u, lr, 0, gpu)
    assert info["validated"] == 0 and info["near_ties"] == 1


def test_reflected_tie_followed_through_passes():
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    f = L.f_coll + 1                 # the crossing interval: a tie
    xm = _mirrored(ref[0], L, f)
    assert not np.allclose(xm, ref[0][L.edges(f)])   # really the other candidate
    _, gpu = _run(inst, override=([f], xm.ravel(), [O.STD]))
    gpu[0] = ref[0].copy()
    gpu[0][L.edges(f)] = xm
    info = compare_iteration(inst, z, u, lr, 0, gpu)
    assert info["validated"] == 1


def test_reflected_tie_not_followed_through_fails():
    """The other candidate on the tie, but z and u as if the first had been
    taken: the consensus check catches it."""
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    f = L.f_coll + 1                 # the crossing interval: a tie
    gpu = [a.copy() for a in ref]
    gpu[0][L.edges(f)] = _mirrored(ref[0], L, f)
    with pytest.raises(AssertionError):
        compare_iteration(inst, z, u, lr, 0, gpu)


def test_infeasible_output_on_a_tie_fails():
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    f = L.f_coll + 1                 # the crossing interval: a tie
    bad = ref[0][L.edges(f)].copy()
    bad[:, 1] *= 0.5                 # halfway back towards the collision
    _, gpu = _run(inst, override=([f], bad.ravel(), [O.STD]))
    gpu[0] = ref[0].copy()
    gpu[0][L.edges(f)] = bad
    with pytest.raises(AssertionError, match="infeasible"):
        compare_iteration(inst, z, u, lr, 0, gpu)


def test_costlier_output_on_a_tie_fails():
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    f = L.f_coll + 1                 # the crossing interval: a tie
    bad = _mirrored(ref[0], L, f)
    bad[:, 1] *= 1.5                 # feasible, but moved further than needed
    _, gpu = _run(inst, override=([f], bad.ravel(), [O.STD]))
    gpu[0] = ref[0].copy()
    gpu[0][L.edges(f)] = bad
    with pytest.raises(AssertionError, match="energy"):
        compare_iteration(inst, z, u, lr, 0, gpu)


def test_difference_away_from_a_tie_fails():
    """An energy factor (closed form, never tied) with a perturbed x."""
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    f = L.f_energy
    gpu = [a.copy() for a in ref]
    gpu[0][L.edges(f)[0], 0] += 1e-3
    with pytest.raises(AssertionError, match="without a near-tie"):
        compare_iteration(inst, z, u, lr, 0, gpu)


def test_wrong_weight_fails():
    inst = _head_on()
    L = Layout(inst)
    (z, u, lr), ref = _run(inst)
    gpu = [a.copy() for a in ref]
    gpu[1][L.f_energy] = O.ZERO
    with pytest.raises(AssertionError):
        compare_iteration(inst, z, u, lr, 0, gpu)


def test_u_error_fails():
    inst = I.random_box(8, 0.06, 3, sigma=2e-2, seed=2, alpha=0.1, C=1 / 24)
    P = O.Planner(inst)
    P.iterate(3)
    z, u, lr = P.get_state()
    z32, u32 = z.astype(np.float32), u.astype(np.float32)
    Q = O.Planner(inst)
    Q.set_state(z32.astype(np.float64), u32.astype(np.float64), lr, 3)
    Q.iterate(1)
    x, rf = Q.last()
    zz, uu, ll = Q.get_state()
    compare_iteration(inst, z32, u32, lr, 3, [x, rf, zz, uu, ll])
    uu = uu.copy()
    uu[len(uu) // 2] += 1e-3
    with pytest.raises(AssertionError):
        compare_iteration(inst, z32, u32, lr, 3, [x, rf, zz, uu, ll])
