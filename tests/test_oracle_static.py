"""Pins for the oracle's static geometry terms (CPU only): fixed oriented
boxes and self-collision between listed link pairs of an arm.

The box term is tied to brute-force sampling of the box surface in world
coordinates (which fixes the axis convention independently of the oracle's
projection), the self term to a hand-derived folded planar arm and to the
rigid-motion invariants of a serial chain.
"""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes


def _bare(d, kind, dh, links, sph, lo, hi, boxes=None, pairs=None):
    return scenes.Problem(
        name="bare", d=d, kind=kind, dh=np.asarray(dh, dtype=np.float64), sphere_link=np.asarray(links, np.int32),
        sphere=np.asarray(sph, dtype=np.float64), q_lo=np.full(d, lo), q_hi=np.full(d, hi),
        q_start=np.zeros(d), q_goal=np.zeros(d), t_min=0.0, t_max=10.0, v_max=1.0,
        n_wp=np.zeros(0, np.int32), wp=np.zeros((0, 1, 4)), obs_r=np.zeros(0),
        self_pairs=np.zeros((0, 2), np.int32) if pairs is None else np.asarray(pairs, np.int32),
        boxes=np.zeros((0, 15)) if boxes is None else np.asarray(boxes, dtype=np.float64))


def _rot(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _surface_points(c, h, axes, n=60):
    """Points on the box surface in world coordinates: c + sum_a u_a axes[a]."""
    g = np.linspace(-1.0, 1.0, n)
    pts = []
    for a in range(3):
        b, e = [k for k in range(3) if k != a]
        U, V = np.meshgrid(g * h[b], g * h[e], indexing="ij")
        for sgn in (-1.0, 1.0):
            loc = np.zeros((U.size, 3))
            loc[:, a] = sgn * h[a]
            loc[:, b] = U.ravel()
            loc[:, e] = V.ravel()
            pts.append(c + loc @ axes)  # row a of axes is the world direction of box axis a
    return np.concatenate(pts)


def test_box_distance_matches_surface_sampling(oracle_lib):
    rng = np.random.default_rng(7)
    for trial in range(12):
        c = rng.uniform(-0.5, 0.5, 3)
        h = rng.uniform(0.05, 0.4, 3)
        axes = _rot(rng)
        r = 0.05
        box = np.concatenate([c, h, axes.ravel()])
        prob = _bare(3, scenes.KIND_TRANSLATE, np.zeros((3, 4)), [0], [[0, 0, 0, r]], -10.0, 10.0, boxes=[box])
        o = oracle_lib.Oracle(prob)
        surf = _surface_points(c, h, axes)
        spacing = 2.0 * h.max() / 59
        for _ in range(20):
            p = c + rng.normal(size=3) * 0.6
            local = axes @ (p - c)
            inside = np.all(np.abs(local) <= h)
            ok, m = o.state_valid(np.concatenate([p, [1.0]]))
            if inside:
                assert not ok and m == pytest.approx(-r, abs=1e-12)
                continue
            dist = np.linalg.norm(surf - p, axis=1).min()   # >= true distance, within the grid spacing
            assert dist - spacing <= m + r <= dist + 1e-12
            if abs(m) > spacing:
                assert ok == (dist >= r)


def test_box_touching_is_free_and_rotation_covariant(oracle_lib):
    # a unit cube turned 45 degrees about z: its corner at +x sits at x = sqrt(2)/2
    s = math.sqrt(0.5)
    axes = np.array([[s, s, 0.0], [-s, s, 0.0], [0.0, 0.0, 1.0]])
    box = np.concatenate([[0, 0, 0], [0.5, 0.5, 0.5], axes.ravel()])
    r = 0.25
    prob = _bare(3, scenes.KIND_TRANSLATE, np.zeros((3, 4)), [0], [[0, 0, 0, r]], -10.0, 10.0, boxes=[box])
    o = oracle_lib.Oracle(prob)
    x = math.sqrt(0.5) + r
    ok, m = o.state_valid(np.array([x, 0.0, 0.0, 1.0]))
    assert ok and abs(m) < 1e-12
    ok, m = o.state_valid(np.array([x - 1e-6, 0.0, 0.0, 1.0]))
    assert not ok
    # along the face normal (1, 1, 0)/sqrt 2 the face is 0.5 away
    ok, m = o.state_valid(np.array([s * 0.8, s * 0.8, 0.0, 1.0]))
    assert ok and m == pytest.approx(0.8 - 0.5 - r, abs=1e-12)


def _planar3(r, pairs):
    # three revolute joints about z, link lengths 1, 0.3, 1; one sphere at each
    # link's midpoint, given in the frame at the link's end
    dh = [[1.0, 0, 0, 0], [0.3, 0, 0, 0], [1.0, 0, 0, 0]]
    sph = [[-0.5, 0, 0, r], [-0.15, 0, 0, r], [-0.5, 0, 0, r]]
    return _bare(3, scenes.KIND_DH, dh, [1, 2, 3], sph, -math.pi, math.pi, pairs=pairs)


def test_self_collision_folded_planar_arm(oracle_lib):
    # q = (0, pi/2, pi/2): link 1 runs (0,0)->(1,0), link 2 (1,0)->(1,0.3),
    # link 3 (1,0.3)->(0,0.3), so the midpoints of links 1 and 3 are 0.3 apart
    q = np.array([0.0, math.pi / 2, math.pi / 2, 0.0])
    for r, expect_ok in ((0.16, False), (0.14, True)):
        o = oracle_lib.Oracle(_planar3(r, [[1, 3]]))
        ok, m = o.state_valid(q)
        assert ok == expect_ok
        assert m == pytest.approx(0.3 - 2 * r, abs=1e-12)
    # the same state with the pair not listed is free (no other term)
    ok, _ = oracle_lib.Oracle(_planar3(0.16, [])).state_valid(q)
    assert ok
    # a listed adjacent pair: midpoints (0.5, 0) and (1, 0.15)
    ok, m = oracle_lib.Oracle(_planar3(0.1, [[1, 2]])).state_valid(q)
    assert ok and m == pytest.approx(math.hypot(0.5, 0.15) - 0.2, abs=1e-12)


@pytest.mark.parametrize("maker", [scenes.arm6, scenes.arm7rr])
def test_self_margin_invariant_to_joints_outside_the_pair(oracle_lib, maker):
    """For one listed pair (la, lb), joints 1..la move both links rigidly and
    joints after lb move neither, so the pair's margin ignores them; a joint
    between the two links changes it."""
    base = maker(0)
    rng = np.random.default_rng(3)
    pairs = scenes.self_pairs_for(base)
    for la, lb in pairs[:6]:
        prob = maker(0)
        prob.n_wp, prob.wp, prob.obs_r = prob.n_wp[:0], prob.wp[:0], prob.obs_r[:0]
        prob.self_pairs = np.array([[la, lb]], np.int32)
        prob.q_lo, prob.q_hi = np.full(prob.d, -50.0), np.full(prob.d, 50.0)
        o = oracle_lib.Oracle(prob)
        q = rng.uniform(-math.pi, math.pi, prob.d)
        _, m0 = o.state_valid(np.concatenate([q, [0.0]]))
        for j in range(prob.d):
            q2 = q.copy()
            q2[j] += 0.7
            _, m1 = o.state_valid(np.concatenate([q2, [0.0]]))
            joint = j + 1        # joint j+1 turns frames j+1 .. d
            if joint <= la or joint > lb:
                assert m1 == pytest.approx(m0, abs=1e-12)


@pytest.mark.parametrize("maker", [scenes.arm6, scenes.arm7rr])
def test_self_pair_tables_are_free_at_home(oracle_lib, maker):
    """The listed pairs are at least two links apart and none touches at
    q = 0; the pairs two or more apart that are left out do touch there."""
    prob = maker(0)
    pairs = scenes.self_pairs_for(prob)
    listed = {tuple(p) for p in pairs.tolist()}
    assert all(b >= a + 2 for a, b in listed)
    prob.n_wp, prob.wp, prob.obs_r = prob.n_wp[:0], prob.wp[:0], prob.obs_r[:0]
    for la in range(1, prob.d + 1):
        for lb in range(la + 2, prob.d + 1):
            prob.self_pairs = np.array([[la, lb]], np.int32)
            ok, m = oracle_lib.Oracle(prob).state_valid(np.zeros(prob.d + 1))
            assert ok == ((la, lb) in listed)
            assert abs(m) > 1e-3


def test_static_geometry_is_time_independent(oracle_lib):
    prob = scenes.with_static(scenes.arm6(5))
    prob.n_wp, prob.wp, prob.obs_r = prob.n_wp[:0], prob.wp[:0], prob.obs_r[:0]
    o = oracle_lib.Oracle(prob)
    rng = np.random.default_rng(11)
    for _ in range(50):
        q = rng.uniform(-math.pi, math.pi, 6)
        a = o.state_valid(np.concatenate([q, [0.5]]))
        b = o.state_valid(np.concatenate([q, [17.0]]))
        assert a == b
