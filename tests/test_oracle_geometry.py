"""Pins for the oracle's geometry, state and edge checks (CPU only).

Each test ties the oracle to something other than itself: hand-derived
forward-kinematics poses, rigid-motion invariants, the closed-form closest
approach of linearly moving discs, and brute-force enumeration on tiny inputs.
"""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes


@pytest.fixture(scope="module")
def ur5e(oracle_lib):
    prob = scenes.arm6(0)
    return oracle_lib.Oracle(prob)


def test_ur5e_zero_pose_hand_derived(ur5e):
    # Standard-DH UR5e at q = 0, derived by hand: the flange origin sits at
    # x = a2 + a3, y = -(d4 + d6), z = d1 - d5.
    fr = ur5e.frames(np.zeros(6))
    expect = np.array([-0.425 - 0.3922, -(0.1333 + 0.0996), 0.1625 - 0.0997])
    assert np.allclose(fr[6][:, 3], expect, atol=2e-7)
    # frame 1 origin at the shoulder height, frame 2 at the end of the upper arm
    assert np.allclose(fr[1][:, 3], [0, 0, 0.1625], atol=1e-7)
    assert np.allclose(fr[2][:, 3], [-0.425, 0, 0.1625], atol=1e-7)
    # the flange z axis points along -y of the base at the zero pose
    assert np.allclose(fr[6][:, 2], [0, -1, 0], atol=1e-7)


def _rodrigues(axis, theta):
    k = axis / np.linalg.norm(axis)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(theta) * K + (1 - math.cos(theta)) * K @ K


@pytest.mark.parametrize("maker", [scenes.arm6, scenes.arm7rr])
def test_joint_rotation_is_rotation_about_joint_axis(oracle_lib, maker):
    prob = maker(3)
    o = oracle_lib.Oracle(prob)
    rng = np.random.default_rng(0)
    for trial in range(6):
        q = rng.uniform(-math.pi, math.pi, size=prob.d)
        i = int(rng.integers(0, prob.d))
        th = float(rng.uniform(-2, 2))
        fr = o.frames(q)
        axis_pt, axis_dir = fr[i][:, 3], fr[i][:, 2]   # joint i+1 turns about z of frame i
        R = _rodrigues(axis_dir, th)
        q2 = q.copy()
        q2[i] += th
        c1, c2 = o.spheres(q), o.spheres(q2)
        for s in range(prob.n_spheres):
            if prob.sphere_link[s] <= i:      # links before the joint do not move
                assert np.allclose(c2[s], c1[s], atol=1e-12)
            else:
                assert np.allclose(c2[s], axis_pt + R @ (c1[s] - axis_pt), atol=1e-12)


def test_rigid_links_keep_sphere_distances(oracle_lib):
    prob = scenes.arm6(1)
    o = oracle_lib.Oracle(prob)
    rng = np.random.default_rng(1)
    c0 = o.spheres(np.zeros(6))
    for _ in range(5):
        c = o.spheres(rng.uniform(-3, 3, 6))
        for l in range(1, 7):
            idx = np.where(prob.sphere_link == l)[0]
            if len(idx) < 2:
                continue
            d0 = np.linalg.norm(c0[idx][:, None] - c0[idx][None], axis=-1)
            d1 = np.linalg.norm(c[idx][:, None] - c[idx][None], axis=-1)
            assert np.allclose(d0, d1, atol=1e-12)


def test_sphere_model_matches_workload(oracle_lib):
    a6, a7 = scenes.arm6(0), scenes.arm7rr(0)
    assert a6.n_spheres == 40 and a7.n_spheres == 60
    assert a6.sphere[:, 3].min() >= 0.03 - 1e-6 and a6.sphere[:, 3].max() <= 0.08 + 1e-6
    assert a6.n_obs == 16 and a6.w_max == 8 and np.allclose(a6.obs_r, 0.1, atol=1e-7)
    assert a7.n_obs == 32 and a7.w_max == 16


def test_obstacle_waypoints_and_constant_velocity(oracle_lib):
    prob = scenes.arm6(2)
    o = oracle_lib.Oracle(prob)
    for ob in range(prob.n_obs):
        for k in range(prob.w_max):
            assert np.allclose(o.obstacle(ob, prob.wp[ob, k, 0]), prob.wp[ob, k, 1:], atol=1e-12)
        # continuity at an interior waypoint
        tk = prob.wp[ob, 3, 0]
        assert np.allclose(o.obstacle(ob, tk - 1e-9), o.obstacle(ob, tk + 1e-9), atol=1e-6)
        # midpoint of a segment is the average of its waypoints
        mid = 0.5 * (prob.wp[ob, 2, 0] + prob.wp[ob, 3, 0])
        assert np.allclose(o.obstacle(ob, mid), 0.5 * (prob.wp[ob, 2, 1:] + prob.wp[ob, 3, 1:]), atol=1e-12)
        # held outside the span
        assert np.allclose(o.obstacle(ob, -5.0), prob.wp[ob, 0, 1:])
        assert np.allclose(o.obstacle(ob, 1e3), prob.wp[ob, -1, 1:])
    disc = scenes.disc2d(0)
    od = oracle_lib.Oracle(disc)
    for ob in range(disc.n_obs):
        c0, c1 = disc.wp[ob, 0, 1:], disc.wp[ob, 1, 1:]
        v = (c1 - c0) / disc.t_max
        for t in [0.0, 1.3, 7.77, 10.0]:
            assert np.allclose(od.obstacle(ob, t), c0 + v * t, atol=1e-12)


def _disc_scene_single(obs_xy0, obs_xy1, r_obs=0.1, r_rob=0.05, H=10.0):
    prob = scenes.disc2d(0)
    prob.n_wp = np.array([2], dtype=np.int32)
    prob.wp = np.array([[[0.0, obs_xy0[0], obs_xy0[1], 0.0], [H, obs_xy1[0], obs_xy1[1], 0.0]]])
    prob.obs_r = np.array([r_obs])
    prob.sphere = np.array([[0.0, 0.0, 0.0, r_rob]])
    prob.t_max = H
    return prob


def test_state_touching_counts_as_free(oracle_lib):
    prob = _disc_scene_single([0.5, 0.5], [0.5, 0.5], r_obs=0.25, r_rob=0.25)
    o = oracle_lib.Oracle(prob)
    # exactly touching (distance 0.5 = 0.25 + 0.25, exact in binary)
    assert o.state_valid([1.0, 0.5, 1.0])[0]
    assert not o.state_valid([0.9999, 0.5, 1.0])[0]
    ok, m = o.state_valid([0.5, 1.0, 2.0])
    assert ok and abs(m) < 1e-15
    # outside the box / horizon
    assert not o.state_valid([1.0 + 1e-9, 0.5, 1.0])[0]
    assert not o.state_valid([0.1, 0.1, -1e-9])[0]
    assert not o.state_valid([0.1, 0.1, prob.t_max + 1e-9])[0]


def _closed_form_dmin(prob, xa, xb):
    """Closest approach of the robot disc and each linearly moving obstacle disc
    over the edge, written out from relative motion p(tau) = p0 + w tau."""
    if xa[2] > xb[2]:
        xa, xb = xb, xa
    T = xb[2] - xa[2]
    best = np.inf
    H = prob.t_max
    for ob in range(prob.n_obs):
        c0, c1 = prob.wp[ob, 0, 1:3], prob.wp[ob, 1, 1:3]
        vo = (c1 - c0) / H
        p0 = xa[:2] - (c0 + vo * xa[2])
        vr = (xb[:2] - xa[:2]) / T if T > 0 else np.zeros(2)
        w = vr - vo if T > 0 else np.zeros(2)
        ww = w @ w
        tau = 0.0 if ww == 0 else min(max(-(p0 @ w) / ww, 0.0), T)
        dist = np.linalg.norm(p0 + w * tau) - (prob.sphere[0, 3] + prob.obs_r[ob])
        best = min(best, dist)
    return best


def test_discrete_edge_check_bracketed_by_closed_form(oracle_lib):
    prob = scenes.disc2d(5)
    o = oracle_lib.Oracle(prob)
    xa, xb = scenes.synthetic_edges(prob, 3000, seed=11, bridge_mix=True)
    xa = xa.astype(np.float64)
    xb = xb.astype(np.float64)
    res = o.check_edges(xa, xb)
    n_free = n_hit = 0
    for e in range(len(xa)):
        dmin = _closed_form_dmin(prob, xa[e], xb[e])
        ok_c, dm_c = o.edge_continuous(xa[e], xb[e])
        assert abs(dm_c - dmin) < 1e-12
        # states visited by the discrete check are a subset of the continuous motion
        if dmin >= 0:
            assert res["free"][e] == 1
            n_free += 1
        # some state is within half a step of the closest approach
        a, b = (xa[e], xb[e]) if xa[e, 2] <= xb[e, 2] else (xb[e], xa[e])
        T = b[2] - a[2]
        vmax_rel = (np.linalg.norm(b[:2] - a[:2]) / T if T > 0 else 0) + 0.2 * math.sqrt(2)
        if dmin < -vmax_rel * T / (2 * res["n"][e]) - 1e-12:
            assert res["free"][e] == 0
            n_hit += 1
    assert n_free > 100 and n_hit > 100


def test_discrete_check_converges_to_continuous(oracle_lib):
    prob = scenes.disc2d(6)
    rng = np.random.default_rng(3)
    xa, xb = scenes.synthetic_edges(prob, 300, seed=12, bridge_mix=True)
    fine = scenes.disc2d(6)
    fine.params.h = prob.params.h / 16
    o, of = oracle_lib.Oracle(prob), oracle_lib.Oracle(fine)
    r1 = o.check_edges(xa, xb)
    r16 = of.check_edges(xa, xb)
    cont = np.array([_closed_form_dmin(prob, xa[e].astype(float), xb[e].astype(float)) >= 0 for e in range(300)])
    # refinement can only find more collisions, and never disagrees with the continuous "free"
    assert np.all(r16["free"] <= r1["free"])
    assert np.all(r16["free"][cont] == 1)
    assert (r16["free"] != cont).sum() <= (r1["free"] != cont).sum()
    del rng


def _piecewise_disc(seed, n_wp=5):
    """disc2d scene whose obstacles follow random 5-waypoint paths."""
    prob = scenes.disc2d(seed)
    rng = np.random.default_rng([7, seed])
    O = prob.n_obs
    wp = np.zeros((O, n_wp, 4))
    times = np.sort(np.r_[0.0, rng.uniform(0.5, 9.5, size=n_wp - 2), 10.0])
    for o in range(O):
        wp[o, :, 0] = times
        wp[o, :, 1:3] = rng.uniform(0.0, 1.0, size=(n_wp, 2))
    prob.wp = scenes.f32(wp)
    prob.n_wp = np.full(O, n_wp, dtype=np.int32)
    return prob


def _sampled_clearance(prob, a, b, n=20001):
    """Brute force: least pair clearance over n evenly spaced times of the
    edge, obstacle positions by linear interpolation of the waypoints."""
    if a[-1] > b[-1]:
        a, b = b, a
    ts = np.linspace(a[-1], b[-1], n)
    f = (ts - a[-1]) / (b[-1] - a[-1]) if b[-1] > a[-1] else np.zeros(n)
    rx = a[0] + f * (b[0] - a[0]) + prob.sphere[0, 0]
    ry = a[1] + f * (b[1] - a[1]) + prob.sphere[0, 1]
    best = np.inf
    for o in range(prob.n_obs):
        w = prob.wp[o, :prob.n_wp[o]]
        ox = np.interp(ts, w[:, 0], w[:, 1])
        oy = np.interp(ts, w[:, 0], w[:, 2])
        oz = np.interp(ts, w[:, 0], w[:, 3])
        dist = np.sqrt((rx - ox) ** 2 + (ry - oy) ** 2 + oz ** 2) - (prob.sphere[0, 3] + prob.obs_r[o])
        best = min(best, dist.min())
    return best


def test_piecewise_continuous_check(oracle_lib):
    """The closed-form check with trajectories cut at their waypoints: equal to
    the single-segment form on constant-velocity scenes; on piecewise scenes
    never above a dense brute-force sampling of the same motion and within
    the sampling resolution of it; consistent with the discrete check (free
    continuously implies free discretely, a discrete hit implies a
    continuous one)."""
    prob = scenes.disc2d(5)
    o = oracle_lib.Oracle(prob)
    xa, xb = scenes.synthetic_edges(prob, 500, seed=13, bridge_mix=True)
    for e in range(len(xa)):
        ok1, d1 = o.edge_continuous(xa[e], xb[e])
        ok2, d2 = o.edge_continuous_pw(xa[e], xb[e])
        assert abs(d1 - d2) < 1e-12 and ok1 == ok2
    pw = _piecewise_disc(8)
    op = oracle_lib.Oracle(pw)
    xa, xb = scenes.synthetic_edges(pw, 400, seed=14, bridge_mix=True)
    xa, xb = xa.astype(np.float64), xb.astype(np.float64)
    res = op.check_edges(xa, xb)
    n_free = n_hit = 0
    for e in range(len(xa)):
        ok, dm = op.edge_continuous_pw(xa[e], xb[e])
        ds = _sampled_clearance(pw, xa[e], xb[e])
        assert ds >= dm - 1e-9, (e, ds, dm)
        assert ds - dm <= 2e-4, (e, ds, dm)
        if ok:
            assert res["free"][e] == 1
            n_free += 1
        if res["free"][e] == 0:
            assert not ok
            n_hit += 1
    assert n_free > 50 and n_hit > 50


def test_edge_check_brute_force_tiny(oracle_lib):
    """Every state x every pair, no early exit, enumerated independently."""
    prob = scenes.arm6(4, n_obs=2, n_wp=3)
    prob.sphere = prob.sphere[[3, 17]]
    prob.sphere_link = prob.sphere_link[[3, 17]]
    o = oracle_lib.Oracle(prob)
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(300):
        xa = np.r_[rng.uniform(-3, 3, 6), rng.uniform(0, 20)]
        step = rng.normal(size=6)
        step *= rng.uniform(0.01, 0.12) / np.linalg.norm(step)
        xb = np.r_[np.clip(xa[:6] + step, -math.pi, math.pi), xa[6] + rng.uniform(0.01, 0.05)]
        res = o.check_edges(xa[None], xb[None])
        n = int(res["n"][0])
        if n > 8:
            continue
        checked += 1
        hits = []
        for j in range(n + 1):
            x = xa + (j / n) * (xb - xa)
            c = o.spheres(x[:6])
            bad = False
            for ob in range(prob.n_obs):
                co = o.obstacle(ob, x[6])
                for s in range(2):
                    if np.linalg.norm(c[s] - co) < prob.sphere[s, 3] + prob.obs_r[ob]:
                        bad = True
            if np.any(x[:6] < prob.q_lo) or np.any(x[:6] > prob.q_hi):
                bad = True
            if bad:
                hits.append(j)
        assert res["free"][0] == (len(hits) == 0)
        assert res["first_hit"][0] == (hits[0] if hits else -1)
        # n follows max(D, v dt) / h
        D = np.linalg.norm(xb[:6] - xa[:6])
        assert n == max(1, math.ceil(max(D, prob.v_max * (xb[6] - xa[6])) / prob.params.h))
    assert checked > 50


def test_edge_check_endpoint_order_invariant(oracle_lib):
    prob = scenes.arm6(7)
    o = oracle_lib.Oracle(prob)
    xa, xb = scenes.synthetic_edges(prob, 400, seed=3)
    r1 = o.check_edges(xa, xb)
    r2 = o.check_edges(xb, xa)
    for k in ("free", "first_hit", "n"):
        assert np.array_equal(r1[k], r2[k])
