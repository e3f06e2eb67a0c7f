"""Pins of the FP64 reference minimisers against closed forms, hand-derived
examples and brute-force constrained minimisation (no GPU)."""
import numpy as np
import pytest

import oracle as O
from tests import bruteforce as bf

INF = np.inf


# ------------------------------------------------------------------ geometry

def test_cpa_matches_sampling():
    rng = np.random.default_rng(0)
    for dim in (2, 3):
        for _ in range(50):
            d0, d1 = rng.normal(size=dim), rng.normal(size=dim)
            assert abs(O.cpa(d0, d1) - bf.cpa_sampled(d0, d1)) < 1e-9


def test_cpa_special_cases():
    # parallel relative motion: distance constant
    assert O.cpa([1, 2], [1, 2]) == pytest.approx(np.sqrt(5), abs=1e-15)
    # head-on through the origin: zero
    assert O.cpa([-1, 0], [1, 0]) == pytest.approx(0, abs=1e-15)
    # passes at height 0.3
    assert O.cpa([-1, 0.3], [1, 0.3]) == pytest.approx(0.3, abs=1e-15)
    # closest point at an end
    assert O.cpa([2, 0], [3, 0]) == pytest.approx(2, abs=1e-15)


def test_segseg_matches_sampling():
    rng = np.random.default_rng(1)
    for _ in range(30):
        p = rng.normal(size=(4, 2))
        want = bf.segseg_exact(*p)
        assert abs(O.segseg(*p) - want) < 1e-7
        assert abs(bf.segseg_closed(*p) - want) < 1e-7
    # crossing segments
    assert O.segseg([-1, 0], [1, 0], [0, -1], [0, 1]) == 0.0


# ------------------------------------------------------------------ energy (App. E)

def test_energy_worked_value():
    # rho_lo = rho_hi = C = 1 gives x_lo = (3 n_lo + 2 n_hi)/5, x_hi = (2 n_lo + 3 n_hi)/5
    nl, nh = np.array([0.3, -1.2]), np.array([2.0, 0.7])
    xl, xh = O.prox_energy(nl, nh, 1.0, 1.0, 1.0)
    assert np.allclose(xl, (3 * nl + 2 * nh) / 5, atol=1e-15)
    assert np.allclose(xh, (2 * nl + 3 * nh) / 5, atol=1e-15)


def test_energy_first_order_conditions():
    """x minimises C|xl-xh|^2 + wl/2|xl-nl|^2 + wh/2|xh-nh|^2: solve the 2x2
    linear system of its gradient directly."""
    rng = np.random.default_rng(2)
    for _ in range(40):
        nl, nh = rng.normal(size=3), rng.normal(size=3)
        wl, wh, C = rng.uniform(0.01, 5, size=3)
        A = np.array([[2 * C + wl, -2 * C], [-2 * C, 2 * C + wh]])
        sol = np.linalg.solve(A, np.stack([wl * nl, wh * nh]))
        xl, xh = O.prox_energy(nl, nh, wl, wh, C)
        assert np.allclose(xl, sol[0], atol=1e-12) and np.allclose(xh, sol[1], atol=1e-12)


def test_energy_limits():
    nl, nh = np.array([1.0, 2.0]), np.array([-3.0, 0.5])
    C, wh = 0.7, 1.3
    # certain lower end: x_lo = n_lo, x_hi minimises C|n_lo-x|^2 + wh/2|x-nh|^2
    xl, xh = O.prox_energy(nl, nh, INF, wh, C)
    assert np.allclose(xl, nl) and np.allclose(xh, (2 * C * nl + wh * nh) / (2 * C + wh), atol=1e-15)
    xl, xh = O.prox_energy(nl, nh, wh, INF, C)
    assert np.allclose(xh, nh) and np.allclose(xl, (2 * C * nh + wh * nl) / (2 * C + wh), atol=1e-15)
    # equal weights tending to zero: both at the midpoint
    xl, xh = O.prox_energy(nl, nh, 0.0, 0.0, C)
    assert np.allclose(xl, 0.5 * (nl + nh)) and np.allclose(xh, 0.5 * (nl + nh))
    # large finite weight approaches the limit
    xl2, xh2 = O.prox_energy(nl, nh, 1e12, wh, C)
    xl, xh = O.prox_energy(nl, nh, INF, wh, C)
    assert np.allclose(xl2, xl, atol=1e-9) and np.allclose(xh2, xh, atol=1e-9)


# ------------------------------------------------------------------ agent-agent (App. C, I)

def test_coll_head_on_worked_example():
    """Two agents of radius 1/4 swap along the x axis in one segment, all
    weights 1.  Difference variables: m_lo = (2,0), m_hi = (-2,0), weight
    1/2 each, R = 1/2.  The tangent family E(theta) = 1/4 (1/2 - 2cos)^2 +
    1/4 (1/2 + 2cos)^2 = 1/8 + 2cos^2 is minimal (1/8) at theta = pi/2 and
    3pi/2 (a tie; the smaller angle is kept).  The slab is y = 1/2 in the
    difference frame, so every agent moves 1/4 sideways."""
    act, xl, xh, xlp, xhp, kind, th = O.prox_coll([-1, 0], [1, 0], [1, 0], [-1, 0], 1, 1, 1, 1, 0.5)
    assert act and kind == 0
    assert th == pytest.approx(np.pi / 2, abs=1e-12)
    assert np.allclose(xl, [-1, -0.25], atol=1e-14) and np.allclose(xh, [1, -0.25], atol=1e-14)
    assert np.allclose(xlp, [1, 0.25], atol=1e-14) and np.allclose(xhp, [-1, 0.25], atol=1e-14)
    E = 0.5 * sum(np.sum((a - b) ** 2) for a, b in zip((xl, xh, xlp, xhp), ([-1, 0], [1, 0], [1, 0], [-1, 0])))
    assert E == pytest.approx(0.125, abs=1e-14)


def test_coll_inactive_returns_n():
    n = [[0, 0], [1, 0], [0, 1], [1, 1]]
    act, *x, kind, th = O.prox_coll(*n, 1, 1, 1, 1, 0.99)
    assert not act and all(np.array_equal(a, b) for a, b in zip(x, np.array(n, float)))
    # exactly touching is feasible (non-strict inequality)
    act, *_ = O.prox_coll(*n, 1, 1, 1, 1, 1.0)
    assert not act


def _coll_energy(x, n, w):
    return 0.5 * sum(wk * np.sum((xk - nk) ** 2) for xk, nk, wk in zip(x, n, w))


@pytest.mark.parametrize("seed", range(6))
def test_coll_vs_bruteforce_equal_weights(seed):
    rng = np.random.default_rng(100 + seed)
    checked = 0
    while checked < 5:
        n = rng.normal(0, 0.35, size=(4, 2))
        R = 0.5
        w = [1.0, 1.0, 1.0, 1.0]
        act, xl, xh, xlp, xhp, kind, th = O.prox_coll(*n, *w, R)
        if not act:
            continue
        x = [xl, xh, xlp, xhp]
        E = _coll_energy(x, n, w)
        assert bf.cpa_np(xlp - xl, xhp - xh) >= R - 1e-12
        best = bf.brute_coll(n, w, R, rng, starts=30)
        assert E <= best[0] * (1 + 1e-7) + 1e-13
        # the brute force is a true local optimum, so it cannot beat the reference by more than its tolerance
        assert E >= best[0] - 1e-7
        # equal weights keep each pair's midpoint
        assert np.allclose(xl + xlp, n[0] + n[2], atol=1e-12) and np.allclose(xh + xhp, n[1] + n[3], atol=1e-12)
        checked += 1


@pytest.mark.parametrize("seed", range(4))
def test_coll_vs_bruteforce_unequal_weights(seed):
    """Unequal weights exercise the re-derived reduction of App. C:
    omega = rho rho'/(rho + rho') and target n' - n."""
    rng = np.random.default_rng(200 + seed)
    checked = 0
    while checked < 4:
        n = rng.normal(0, 0.35, size=(4, 2))
        R = 0.5
        w = rng.uniform(0.2, 4.0, size=4)
        act, xl, xh, xlp, xhp, kind, th = O.prox_coll(*n, *w, R)
        if not act:
            continue
        E = _coll_energy([xl, xh, xlp, xhp], n, w)
        best = bf.brute_coll(n, w, R, rng, starts=30)
        assert bf.cpa_np(xlp - xl, xhp - xh) >= R - 1e-12
        assert abs(E - best[0]) <= 1e-7 * max(1.0, best[0])
        checked += 1


def test_coll_certain_lower_end_vs_bruteforce():
    """Weight infinity on both lower ends (first segment, whose start is
    fixed): the lower ends stay, only the upper ends move."""
    rng = np.random.default_rng(7)
    checked = 0
    while checked < 6:
        n = rng.normal(0, 0.4, size=(4, 2))
        R = 0.3
        if np.linalg.norm(n[2] - n[0]) < R:  # the fixed ends must be feasible
            continue
        act, xl, xh, xlp, xhp, kind, th = O.prox_coll(*n, INF, 1.0, INF, 1.0, R)
        if not act:
            continue
        assert np.array_equal(xl, n[0]) and np.array_equal(xlp, n[2])
        E = 0.5 * (np.sum((xh - n[1]) ** 2) + np.sum((xhp - n[3]) ** 2))
        best = bf.brute_coll(n, [1e7, 1.0, 1e7, 1.0], R, rng, starts=30)
        assert bf.cpa_np(xlp - xl, xhp - xh) >= R - 1e-12
        assert E <= best[0] * (1 + 1e-5) + 1e-10
        assert E >= best[0] - 1e-5
        checked += 1


def test_coll_3d_vs_bruteforce():
    rng = np.random.default_rng(11)
    checked = 0
    while checked < 6:
        n = rng.normal(0, 0.35, size=(4, 3))
        R = 0.5
        w = [1.0, 1.0, 1.0, 1.0]
        act, xl, xh, xlp, xhp, kind, th = O.prox_coll(*n, *w, R)
        if not act:
            continue
        E = _coll_energy([xl, xh, xlp, xhp], n, w)
        best = bf.brute_coll(n, w, R, rng, starts=30)
        assert bf.cpa_np(xlp - xl, xhp - xh) >= R - 1e-12
        assert abs(E - best[0]) <= 1e-7 * max(1.0, best[0])
        checked += 1


def test_coll_planar_3d_equals_2d():
    """A 3-D instance lying in the plane z = 0 gives the 2-D answer."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        n = rng.normal(0, 0.35, size=(4, 2))
        a2 = O.prox_coll(*n, 1, 1, 1, 1, 0.5)
        n3 = np.concatenate([n, np.zeros((4, 1))], axis=1)
        a3 = O.prox_coll(*n3, 1, 1, 1, 1, 0.5)
        assert a2[0] == a3[0]
        for k in range(1, 5):
            assert np.allclose(a3[k][:2], a2[k], atol=1e-12) and abs(a3[k][2]) < 1e-12


def test_coll_energy_equals_separating_scan():
    """The reference's energy equals the 1-D separating-line formulation of
    the disk problem on the difference variables (independent derivation)."""
    rng = np.random.default_rng(13)
    checked = 0
    while checked < 25:
        n = rng.normal(0, 0.35, size=(4, 2))
        w = rng.uniform(0.3, 3.0, size=4)
        R = 0.5
        act, xl, xh, xlp, xhp, kind, th = O.prox_coll(*n, *w, R)
        if not act:
            continue
        E = _coll_energy([xl, xh, xlp, xhp], n, w)
        om = [w[0] * w[2] / (w[0] + w[2]), w[1] * w[3] / (w[1] + w[3])]
        m = np.stack([n[2] - n[0], n[3] - n[1]])
        Es = bf.separating_scan([0, 0], [0, 0], R, m, om)
        assert abs(E - Es) <= 1e-9 * max(Es, 1e-12)
        checked += 1


# ------------------------------------------------------------------ agent-wall (App. D, I)

def _wall_case(rng):
    c = rng.uniform(-0.3, 0.3, 2)
    th = rng.uniform(0, np.pi)
    L = rng.uniform(0.0, 0.8)
    h = 0.5 * L * np.array([np.cos(th), np.sin(th)])
    return c - h, c + h


@pytest.mark.parametrize("seed", range(5))
def test_capsule_vs_bruteforce(seed):
    rng = np.random.default_rng(300 + seed)
    checked = 0
    while checked < 4:
        xL, xR = _wall_case(rng)
        n = rng.normal(0, 0.5, size=(2, 2))
        r = rng.uniform(0.05, 0.3)
        w = rng.uniform(0.3, 3.0, size=2) if seed % 2 else np.ones(2)
        act, x0, x1, kind, th = O.prox_capsule(xL, xR, r, n[0], n[1], *w)
        if not act:
            continue
        E = 0.5 * (w[0] * np.sum((x0 - n[0]) ** 2) + w[1] * np.sum((x1 - n[1]) ** 2))
        assert bf.segseg_closed(x0, x1, xL, xR) >= r - 1e-9
        best = bf.brute_capsule(xL, xR, r, n, w, rng, starts=30)
        assert E <= best[0] * (1 + 1e-7) + 1e-12
        assert E >= best[0] - 1e-6
        checked += 1


def test_capsule_energy_equals_separating_scan():
    rng = np.random.default_rng(14)
    checked = 0
    kinds = set()
    while checked < 60:
        xL, xR = _wall_case(rng)
        n = rng.normal(0, 0.5, size=(2, 2))
        r = rng.uniform(0.05, 0.3)
        w = rng.uniform(0.3, 3.0, size=2)
        act, x0, x1, kind, th = O.prox_capsule(xL, xR, r, n[0], n[1], *w)
        if not act:
            continue
        kinds.add(kind)
        E = 0.5 * (w[0] * np.sum((x0 - n[0]) ** 2) + w[1] * np.sum((x1 - n[1]) ** 2))
        Es = bf.separating_scan(xL, xR, r, n, w)
        assert abs(E - Es) <= 1e-8 * max(Es, 1e-12), (xL, xR, r, n, w, kind)
        checked += 1
    assert {0, 1, 2} <= kinds  # tangent and both boundary scenarios occurred


def test_capsule_degenerate_is_disk():
    """x_L == x_R is a disk: the wall minimiser on n equals the coll
    minimiser's difference variables when the second agent sits at rest
    with infinite weight at the disk centre."""
    rng = np.random.default_rng(15)
    for _ in range(20):
        c = rng.normal(0, 0.2, 2)
        n = rng.normal(0, 0.4, size=(2, 2))
        r = 0.3
        a = O.prox_capsule(c, c, r, n[0], n[1], 1.0, 1.0)
        b = O.prox_coll(n[0], n[1], c, c, 1.0, 1.0, INF, INF, r)
        assert a[0] == b[0]
        if a[0]:
            assert np.allclose(a[1], b[1], atol=1e-10) and np.allclose(a[2], b[2], atol=1e-10)


def test_capsule_certain_end():
    rng = np.random.default_rng(16)
    checked = 0
    while checked < 8:
        xL, xR = _wall_case(rng)
        n = rng.normal(0, 0.5, size=(2, 2))
        r = 0.15
        if bf.point_seg(n[0], xL, xR) < r:
            continue
        act, x0, x1, kind, th = O.prox_capsule(xL, xR, r, n[0], n[1], INF, 1.0)
        if not act:
            continue
        assert np.array_equal(x0, n[0])
        E = 0.5 * np.sum((x1 - n[1]) ** 2)
        assert bf.segseg_closed(x0, x1, xL, xR) >= r - 1e-9
        best = bf.brute_capsule(xL, xR, r, n, [1e7, 1.0], rng, starts=30)
        assert E <= best[0] * (1 + 1e-5) + 1e-10
        checked += 1


# ------------------------------------------------------------------ velocity limits (App. F, G)

@pytest.mark.parametrize("minimum", [False, True])
def test_velocity_minimiser_vs_bruteforce(minimum):
    rng = np.random.default_rng(40 + minimum)
    checked = 0
    for _ in range(60):
        dim = int(rng.choice([2, 3]))
        nl, nh = rng.normal(0, 1, dim), rng.normal(0, 1, dim)
        wl, wh = rng.uniform(0.2, 3.0, 2)
        d = np.linalg.norm(nl - nh)
        C = d * rng.uniform(1.2, 2.5) if minimum else d * rng.uniform(0.2, 0.8)
        act, xl, xh = O.prox_vel(nl, nh, wl, wh, C, minimum)
        assert act
        bl, bh, bf_val = bf.brute_vel(nl, nh, wl, wh, C, minimum, seed=checked)
        val = 0.5 * wl * np.sum((xl - nl) ** 2) + 0.5 * wh * np.sum((xh - nh) ** 2)
        assert abs(np.linalg.norm(xl - xh) - C) < 1e-9 * max(C, 1)
        assert val <= bf_val + 1e-8 * max(bf_val, 1e-8)
        assert np.allclose(xl, bl, atol=1e-5) and np.allclose(xh, bh, atol=1e-5)
        checked += 1
    assert checked == 60


@pytest.mark.parametrize("minimum", [False, True])
def test_velocity_minimiser_inactive_keeps_n(minimum):
    nl, nh = np.array([0.2, -0.1]), np.array([0.5, 0.3])  # distance 0.5
    C = 0.3 if minimum else 0.7
    act, xl, xh = O.prox_vel(nl, nh, 1.0, 2.0, C, minimum)
    assert not act and np.array_equal(xl, nl) and np.array_equal(xh, nh)


def test_velocity_minimiser_weighted_mean_and_certain_end():
    nl, nh = np.array([0.0, 0.0]), np.array([3.0, 4.0])
    # equal weights: the midpoint stays, the ends move symmetrically to distance C
    act, xl, xh = O.prox_vel(nl, nh, 1.0, 1.0, 2.0, False)
    assert np.allclose(0.5 * (xl + xh), [1.5, 2.0]) and np.allclose(xh - xl, [1.2, 1.6])
    # unequal: the weighted mean stays
    act, xl, xh = O.prox_vel(nl, nh, 1.0, 3.0, 2.0, False)
    assert np.allclose((1.0 * xl + 3.0 * xh) / 4.0, (1.0 * nl + 3.0 * nh) / 4.0)
    # a certain lower end: the upper end is projected onto the circle of radius C around it
    act, xl, xh = O.prox_vel(nl, nh, np.inf, 1.0, 2.0, False)
    assert np.array_equal(xl, nl) and np.allclose(xh, [1.2, 1.6])
    act, xl, xh = O.prox_vel(nl, nh, 1.0, np.inf, 10.0, True)
    assert np.array_equal(xh, nh) and np.allclose(xl, [-3.0, -4.0])
    # large finite weight approaches the certain-end limit
    act, xl2, xh2 = O.prox_vel(nl, nh, 1.0, 1e9, 10.0, True)
    assert np.allclose(xl2, xl, atol=1e-6)


def test_minimum_velocity_coinciding_ends():
    p = np.array([0.4, -0.2])
    act, xl, xh = O.prox_vel(p, p, 1.0, 3.0, 2.0, True)
    assert act and np.allclose(xl - xh, [2.0, 0.0]) and np.allclose((xl + 3 * xh) / 4, p)


def _golden_rows(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        w = lambda t: np.inf if t == "inf" else float(t)
        yield dict(kind=tok[0], wl=w(tok[1]), wh=w(tok[2]), C=float(tok[3]),
                   nl=np.array([float(tok[4]), float(tok[5])]), nh=np.array([float(tok[6]), float(tok[7])]),
                   xl=np.array([float(tok[8]), float(tok[9])]), xh=np.array([float(tok[10]), float(tok[11])]),
                   binding=tok[12] == "1", src=" ".join(tok[13:]))


def test_closed_forms_match_hand_worked_values():
    """tests/golden/closed_forms.txt: energy (App. E), maximum and minimum
    velocity (App. F, G) minimisers on hand-derived exact cases."""
    rows = list(_golden_rows("closed_forms.txt"))
    assert len(rows) >= 9
    for r in rows:
        if r["kind"] == "energy":
            xl, xh = O.prox_energy(r["nl"], r["nh"], r["wl"], r["wh"], r["C"])
            binding = True
        else:
            binding, xl, xh = O.prox_vel(r["nl"], r["nh"], r["wl"], r["wh"], r["C"], r["kind"] == "minvel")
        assert binding == r["binding"], r["src"]
        assert np.allclose(xl, r["xl"], atol=1e-12) and np.allclose(xh, r["xh"], atol=1e-12), (r["src"], xl, xh)
