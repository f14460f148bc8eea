"""Seeded synthetic planning problems (data only).

This module builds the inputs that both the HIP path and the FP64 test oracle
consume: robot tables, obstacle waypoint tables, start/goal configurations and
planner parameters.  It holds none of the planner's arithmetic (no forward
kinematics, no collision tests, no distances); problems are not filtered for
validity here, callers decide what an invalid start or goal means.

Every floating-point value is rounded to the nearest FP32 number and stored as
FP64, so the FP32 device path and the FP64 oracle read identical inputs.

Workloads (the paper's suites are not available, these stand in for them with
the shapes the paper's evaluation uses, Sec. VI Table I):

* ``disc2d``  - disc robot of radius 0.05 in the unit square, 8 disc obstacles
  of radius 0.08 moving at constant velocity (speed <= 0.2), horizon 10 s,
  v_max 1, arrival range [2, 10], interval root with 4 groups, 256 samples per
  iteration, edge step 0.01.
* ``arm6``    - 6-DOF UR5e-like arm (standard DH) as 40 spheres of radius
  0.03-0.08 m, 16 sphere obstacles of radius 0.1 m on piecewise-linear
  trajectories with 8 waypoints in a 1 m cube, joint speed limit 3.14 rad/s,
  arrival range [2, 20], interval root with 8 groups, 4096 samples, step
  0.02 rad.
* ``arm7rr``  - 7-DOF arm as 60 spheres, 32 obstacles of radius 0.05-0.15 m on
  16-waypoint trajectories, arrival range [1, 60], root recycling with 64
  slots, 8192 samples.
* ``mixed``   - heterogeneous problems (DOF 2, 6 or 7; 4-64 obstacles; arrival
  widths 5-60 s; tree capacity 2^14-2^18) for the batched launch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Robot kinds.
KIND_TRANSLATE = 0  # sphere centre = (q0, q1[, q2]) + local offset
KIND_DH = 1         # standard Denavit-Hartenberg serial chain

VARIANT_IR = 0  # interval root (Sec. IV-B, Alg. 2)
VARIANT_RR = 1  # root recycling (Sec. V, Alg. 3)

MAX_DOF = 7


def f32(x):
    """Round to the nearest FP32 value, returned as FP64 (scalar or array)."""
    if np.isscalar(x):
        return float(np.float32(x))
    return np.asarray(x, dtype=np.float32).astype(np.float64)


@dataclass
class Params:
    variant: int = VARIANT_IR
    n_groups: int = 4          # N: interval-root groups or recycling slots
    batch: int = 256           # B: samples (workers) per iteration
    eta: float = 0.1           # steering range
    h: float = 0.01            # edge discretisation step
    dt: float = 0.02           # environment time step (goal grid spacing)
    p_new: float = 0.05
    p_guided: float = 0.95
    cap_fwd: int = 1 << 16     # forward-tree capacity (nodes)
    cap_bwd: int = 1 << 14     # capacity of each backward pool (group or slot)
    seed: int = 1
    no_recycling: int = 0      # recycling variant: keep the initial roots (the paper's ablation)
    obstacle_tile: int = 0     # collision kernels' obstacle tile: 0 automatic, or 4 / 8 / 16


@dataclass
class Problem:
    name: str
    d: int
    kind: int
    dh: np.ndarray            # (d, 4): a, alpha, d_offset, theta0
    sphere_link: np.ndarray   # (S,) int32: 0 = base frame, l = frame after joint l
    sphere: np.ndarray        # (S, 4): local x, y, z, radius
    q_lo: np.ndarray
    q_hi: np.ndarray
    q_start: np.ndarray
    q_goal: np.ndarray
    t_min: float
    t_max: float
    v_max: float
    n_wp: np.ndarray          # (O,) int32
    wp: np.ndarray            # (O, Wmax, 4): t, x, y, z
    obs_r: np.ndarray         # (O,)
    params: Params = field(default_factory=Params)
    seed: int = 0
    # static geometry of arms: link pairs (la, lb) whose spheres are tested
    # against each other, and fixed oriented boxes, one row each: centre (3),
    # half extents (3), unit box axes in world coordinates (3 x 3, row-major)
    self_pairs: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), dtype=np.int32))
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 15), dtype=np.float64))

    @property
    def n_spheres(self) -> int:
        return int(self.sphere.shape[0])

    @property
    def n_obs(self) -> int:
        return int(self.obs_r.shape[0])

    @property
    def w_max(self) -> int:
        return int(self.wp.shape[1])


# ----------------------------------------------------------------------------
# Robot tables
# ----------------------------------------------------------------------------

# UR5e standard DH constants as published by Universal Robots (a, alpha, d).
UR5E_DH = np.array([
    [0.0,     math.pi / 2, 0.1625, 0.0],
    [-0.425,  0.0,         0.0,    0.0],
    [-0.3922, 0.0,         0.0,    0.0],
    [0.0,     math.pi / 2, 0.1333, 0.0],
    [0.0,    -math.pi / 2, 0.0997, 0.0],
    [0.0,     0.0,         0.0996, 0.0],
])

# A fixed 7-DOF standard-DH table with Panda-like link lengths.
ARM7_DH = np.array([
    [0.0,     -math.pi / 2, 0.333, 0.0],
    [0.0,      math.pi / 2, 0.0,   0.0],
    [0.0825,   math.pi / 2, 0.316, 0.0],
    [-0.0825, -math.pi / 2, 0.0,   0.0],
    [0.0,      math.pi / 2, 0.384, 0.0],
    [0.088,    math.pi / 2, 0.0,   0.0],
    [0.0,      0.0,         0.107, 0.0],
])


# Self-collision link pairs.  Reading: the pairs at least two links apart
# whose sphere models do not touch at q = 0 (pairs that touch in that pose,
# and neighbouring links, which share a joint, are left out, as an
# allowed-collision list built from the home pose would).
UR5E_SELF_PAIRS = np.array([[1, 3], [1, 4], [1, 5], [1, 6], [2, 4], [2, 5], [2, 6], [3, 5], [3, 6], [4, 6]],
                           dtype=np.int32)
ARM7_SELF_PAIRS = np.array([[1, 4], [1, 5], [1, 6], [1, 7], [2, 4], [2, 5], [2, 6], [2, 7], [3, 6], [3, 7],
                            [4, 6], [4, 7], [5, 7]], dtype=np.int32)


def _box(centre, half, yaw=0.0):
    """Box row: centre, half extents, unit axes (rows) after a turn about z."""
    c, s = math.cos(yaw), math.sin(yaw)
    axes = np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])
    return np.concatenate([np.asarray(centre, dtype=np.float64), np.asarray(half, dtype=np.float64), axes.ravel()])


# Static environment of the arm workloads with fixed geometry: a table whose
# top lies 7 cm below the base frame (clear of the base spheres) and a post
# turned 30 degrees about z beside the robot.
STATIC_BOXES = np.stack([
    _box([0.0, 0.0, -0.095], [0.9, 0.9, 0.025]),
    _box([0.55, 0.25, 0.3], [0.05, 0.15, 0.3], yaw=math.pi / 6),
])


def _link_segment_in_own_frame(a, alpha, dd):
    """Start point of link i's segment expressed in frame i.

    The link runs from the origin of frame i-1 to the origin of frame i; under
    the standard DH convention the former sits at (-a, -d sin(alpha),
    -d cos(alpha)) in frame i, independent of the joint angle.
    """
    return np.array([-a, -dd * math.sin(alpha), -dd * math.cos(alpha)])


def arm_spheres(dh: np.ndarray, n_spheres: int, r_base: float, r_tip: float):
    """Spread ``n_spheres`` spheres along the link segments at equal arc length.

    Every link gets at least one sphere; the rest are shared in proportion to
    the segment lengths.  Radii fall linearly from ``r_base`` to ``r_tip``
    with cumulative arc length.
    """
    d = dh.shape[0]
    starts = [_link_segment_in_own_frame(dh[i, 0], dh[i, 1], dh[i, 2]) for i in range(d)]
    lengths = np.array([np.linalg.norm(s) for s in starts])
    extra = n_spheres - d
    assert extra >= 0
    share = lengths / max(lengths.sum(), 1e-12) * extra
    counts = np.floor(share).astype(int)
    rem = extra - counts.sum()
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rem]] += 1
    counts += 1
    total = lengths.sum()
    links, xyzr = [], []
    cum = 0.0
    for i in range(d):
        k = counts[i]
        for j in range(k):
            s = (j + 0.5) / k                    # fraction along the segment
            p = starts[i] * (1.0 - s)            # from frame i-1 origin toward frame i origin
            arc = (cum + s * lengths[i]) / max(total, 1e-12)
            r = r_base + (r_tip - r_base) * arc
            links.append(i + 1)
            xyzr.append([p[0], p[1], p[2], r])
        cum += lengths[i]
    return np.array(links, dtype=np.int32), f32(np.array(xyzr))


# ----------------------------------------------------------------------------
# Obstacles
# ----------------------------------------------------------------------------

def _uniform_waypoint_times(h, w):
    return np.array([k * h / (w - 1) for k in range(w)])


def _cube_point(rng, base_r=0.15):
    while True:
        x, y = rng.uniform(-0.5, 0.5, size=2)
        if x * x + y * y >= base_r * base_r:
            return np.array([x, y, rng.uniform(0.0, 1.0)])


def sphere_obstacles(rng, n_obs, n_wp, horizon, radii):
    wp = np.zeros((n_obs, n_wp, 4))
    times = _uniform_waypoint_times(horizon, n_wp)
    for o in range(n_obs):
        for k in range(n_wp):
            wp[o, k, 0] = times[k]
            wp[o, k, 1:] = _cube_point(rng)
    return np.full(n_obs, n_wp, dtype=np.int32), f32(wp), f32(np.asarray(radii, dtype=np.float64))


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

def _pair_rng(rng, kind: int, seed: int, attempt: int):
    """Random stream of the start/goal draw: attempt 0 continues the
    problem's own stream (after the obstacles), attempt k > 0 is a separate
    stream, so a problem can be redrawn keeping its obstacles."""
    return rng if attempt == 0 else np.random.default_rng([0x5EED, kind, seed, 0x57A6, attempt])


def disc2d(seed: int, n_obs: int = 8, horizon: float = 10.0, t_min: float = 2.0,
           params: Params | None = None, attempt: int = 0) -> Problem:
    rng = np.random.default_rng([0x5EED, 1, seed])
    r_robot = 0.05
    wp = np.zeros((n_obs, 2, 4))
    for o in range(n_obs):
        c0 = rng.uniform(0.0, 1.0, size=2)
        heading = rng.uniform(0.0, 2.0 * math.pi)
        speed = rng.uniform(0.0, 0.2)
        v = speed * np.array([math.cos(heading), math.sin(heading)])
        wp[o, 0] = [0.0, c0[0], c0[1], 0.0]
        wp[o, 1] = [horizon, c0[0] + v[0] * horizon, c0[1] + v[1] * horizon, 0.0]
    prng = _pair_rng(rng, 1, seed, attempt)
    while True:
        qs = prng.uniform(r_robot, 1.0 - r_robot, size=2)
        qg = prng.uniform(r_robot, 1.0 - r_robot, size=2)
        if np.linalg.norm(qs - qg) >= 0.5:
            break
    p = params or Params(variant=VARIANT_IR, n_groups=4, batch=256, eta=0.1, h=0.01,
                         cap_fwd=1 << 16, cap_bwd=1 << 14, seed=1)
    return Problem(
        name="disc2d", d=2, kind=KIND_TRANSLATE, dh=np.zeros((2, 4)),
        sphere_link=np.zeros(1, dtype=np.int32), sphere=f32(np.array([[0.0, 0.0, 0.0, r_robot]])),
        q_lo=f32(np.zeros(2)), q_hi=f32(np.ones(2)), q_start=f32(qs), q_goal=f32(qg),
        t_min=f32(t_min), t_max=f32(horizon), v_max=f32(1.0),
        n_wp=np.full(n_obs, 2, dtype=np.int32), wp=f32(wp), obs_r=f32(np.full(n_obs, 0.08)),
        params=p, seed=seed)


def arm6(seed: int, n_obs: int = 16, n_wp: int = 8, horizon: float = 20.0, t_min: float = 2.0,
         params: Params | None = None, attempt: int = 0) -> Problem:
    rng = np.random.default_rng([0x5EED, 2, seed])
    links, sph = arm_spheres(UR5E_DH, 40, 0.08, 0.03)
    n_wp_arr, wp, r = sphere_obstacles(rng, n_obs, n_wp, horizon, np.full(n_obs, 0.1))
    prng = _pair_rng(rng, 2, seed, attempt)
    qs = prng.uniform(-math.pi, math.pi, size=6)
    qg = prng.uniform(-math.pi, math.pi, size=6)
    p = params or Params(variant=VARIANT_IR, n_groups=8, batch=4096, eta=0.5, h=0.02,
                         cap_fwd=1 << 18, cap_bwd=1 << 16, seed=1)
    return Problem(
        name="arm6", d=6, kind=KIND_DH, dh=f32(UR5E_DH), sphere_link=links, sphere=sph,
        q_lo=f32(np.full(6, -math.pi)), q_hi=f32(np.full(6, math.pi)),
        q_start=f32(qs), q_goal=f32(qg), t_min=f32(t_min), t_max=f32(horizon), v_max=f32(3.14),
        n_wp=n_wp_arr, wp=wp, obs_r=r, params=p, seed=seed)


def arm7rr(seed: int, n_obs: int = 32, n_wp: int = 16, horizon: float = 60.0, t_min: float = 1.0,
           params: Params | None = None, attempt: int = 0) -> Problem:
    rng = np.random.default_rng([0x5EED, 3, seed])
    links, sph = arm_spheres(ARM7_DH, 60, 0.08, 0.03)
    radii = rng.uniform(0.05, 0.15, size=n_obs)
    n_wp_arr, wp, r = sphere_obstacles(rng, n_obs, n_wp, horizon, radii)
    prng = _pair_rng(rng, 3, seed, attempt)
    qs = prng.uniform(-math.pi, math.pi, size=7)
    qg = prng.uniform(-math.pi, math.pi, size=7)
    p = params or Params(variant=VARIANT_RR, n_groups=64, batch=8192, eta=0.5, h=0.02,
                         cap_fwd=1 << 18, cap_bwd=1 << 14, seed=1)
    return Problem(
        name="arm7rr", d=7, kind=KIND_DH, dh=f32(ARM7_DH), sphere_link=links, sphere=sph,
        q_lo=f32(np.full(7, -math.pi)), q_hi=f32(np.full(7, math.pi)),
        q_start=f32(qs), q_goal=f32(qg), t_min=f32(t_min), t_max=f32(horizon), v_max=f32(3.14),
        n_wp=n_wp_arr, wp=wp, obs_r=r, params=p, seed=seed)


def mixed(seed: int, attempt: int = 0) -> Problem:
    """One problem of the heterogeneous batch (DOF 2/6/7, 4-64 obstacles)."""
    rng = np.random.default_rng([0x5EED, 4, seed])
    d = int(rng.choice([2, 6, 7]))
    n_obs = int(rng.integers(4, 65))
    width = float(rng.uniform(5.0, 60.0))
    t0 = float(rng.uniform(0.0, 2.0))
    cap_log = int(rng.integers(14, 19))
    sub = int(rng.integers(0, 1 << 30))
    if d == 2:
        p = Params(variant=VARIANT_IR, n_groups=4, batch=64, eta=0.1, h=0.01,
                   cap_fwd=1 << cap_log, cap_bwd=1 << max(cap_log - 2, 10), seed=1)
        return disc2d(sub, n_obs=n_obs, horizon=t0 + width, t_min=t0, params=p, attempt=attempt)
    if d == 6:
        p = Params(variant=VARIANT_IR, n_groups=8, batch=64, eta=0.5, h=0.02,
                   cap_fwd=1 << cap_log, cap_bwd=1 << max(cap_log - 3, 10), seed=1)
        return arm6(sub, n_obs=n_obs, horizon=t0 + width, t_min=t0, params=p, attempt=attempt)
    p = Params(variant=VARIANT_RR, n_groups=16, batch=64, eta=0.5, h=0.02,
               cap_fwd=1 << cap_log, cap_bwd=1 << max(cap_log - 4, 10), seed=1)
    return arm7rr(sub, n_obs=n_obs, horizon=t0 + width, t_min=t0, params=p, attempt=attempt)


def self_pairs_for(prob: Problem) -> np.ndarray:
    """The self-collision link pairs of the problem's arm."""
    if prob.kind != KIND_DH:
        return np.zeros((0, 2), dtype=np.int32)
    return {6: UR5E_SELF_PAIRS, 7: ARM7_SELF_PAIRS}[prob.d].copy()


def with_static(prob: Problem, boxes: np.ndarray | None = None) -> Problem:
    """The arm problem with self-collision and the static boxes switched on
    (the moving obstacles, start and goal unchanged)."""
    assert prob.kind == KIND_DH, "static geometry is defined for arms"
    prob.self_pairs = self_pairs_for(prob)
    prob.boxes = np.array(STATIC_BOXES if boxes is None else boxes, dtype=np.float64).reshape(-1, 15)
    prob.name = prob.name + "-static"
    return prob


def arm6static(seed: int, **kw) -> Problem:
    return with_static(arm6(seed, **kw))


def redraw_until(make, accept, max_attempts: int = 64):
    """The first of make(0), make(1), ... (the same obstacles, start and goal
    drawn again from the attempt's own stream) that accept() takes, and the
    attempt index; (None, max_attempts) if none.  The acceptance test is the
    caller's: this module decides nothing about validity.  Evaluation sets use
    it to keep only problems whose start is free at t = 0 and whose goal is
    free at some goal-grid time, as the paper assumes of its queries."""
    for a in range(max_attempts):
        prob = make(a)
        if accept(prob):
            return prob, a
    return None, max_attempts


WORKLOADS = {"disc2d": disc2d, "arm6": arm6, "arm7rr": arm7rr, "mixed": mixed, "arm6static": arm6static}


# ----------------------------------------------------------------------------
# Synthetic edge and query sets
# ----------------------------------------------------------------------------

def synthetic_edges(prob: Problem, n_edges: int, seed: int, bridge_mix: bool = False):
    """Speed-feasible synthetic edges.

    x_a ~ U(C x [0, H]); direction uniform on the unit sphere of C; length
    D ~ U[0, eta] (or U[0, 4 eta] for the bridge mix), reflected at the box
    faces; t_b = t_a + D / (v u) with u ~ U[0.25, 1], capped at H.  Returns (xa, xb) as FP32 arrays of shape (E, d+1),
    time last.
    """
    rng = np.random.default_rng([0xED9E, seed])
    d = prob.d
    lo, hi = prob.q_lo, prob.q_hi
    qa = rng.uniform(lo, hi, size=(n_edges, d))
    ta = rng.uniform(0.0, prob.t_max, size=n_edges)
    dirs = rng.normal(size=(n_edges, d))
    dirs /= np.maximum(np.linalg.norm(dirs, axis=1, keepdims=True), 1e-12)
    scale = 4.0 if bridge_mix else 1.0
    length = rng.uniform(0.0, prob.params.eta * scale, size=n_edges)
    qb = qa + dirs * length[:, None]
    # reflect at the box faces (clipping would park endpoints exactly on them)
    qb = np.where(qb > hi, 2 * hi - qb, qb)
    qb = np.where(qb < lo, 2 * lo - qb, qb)
    qb = np.clip(qb, lo, hi)
    u = rng.uniform(0.25, 1.0, size=n_edges)
    tb = np.minimum(ta + length / (prob.v_max * u), prob.t_max)
    xa = np.concatenate([qa, ta[:, None]], axis=1).astype(np.float32)
    xb = np.concatenate([qb, tb[:, None]], axis=1).astype(np.float32)
    return xa, xb


def synthetic_states(prob: Problem, n: int, seed: int):
    """States uniform in C x [0, H], FP32 (n, d+1)."""
    rng = np.random.default_rng([0x57A7, seed])
    q = rng.uniform(prob.q_lo, prob.q_hi, size=(n, prob.d))
    t = rng.uniform(0.0, prob.t_max, size=n)
    return np.concatenate([q, t[:, None]], axis=1).astype(np.float32)


def synthetic_tree(prob: Problem, n_nodes: int, seed: int, sigma: int = 1):
    """A random tree for nearest-node tests: nodes uniform in C x [0, H].

    Returns q (n, d), t (n,), parent (n,) int32 (parent index < own index,
    root has -1).  Parent times are not made consistent; the nearest-node scan
    does not look at parents.
    """
    rng = np.random.default_rng([0x7EE, seed])
    q = f32(rng.uniform(prob.q_lo, prob.q_hi, size=(n_nodes, prob.d)))
    t = f32(rng.uniform(0.0, prob.t_max, size=n_nodes))
    parent = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n_nodes)], dtype=np.int32) \
        if n_nodes < 4096 else np.concatenate(
            [[-1], (rng.random(n_nodes - 1) * np.arange(1, n_nodes)).astype(np.int32)]).astype(np.int32)
    return q, t, parent


# ----------------------------------------------------------------------------
# Proposal-network feature rows (input formatting only)
# ----------------------------------------------------------------------------

PROP_CORE = 16           # q_s (7), q_g (7), t_min, t_max
PROP_ENC_IN = 65         # 16 waypoints x (t, x, y, z), radius
PROP_T_SCALE = 60.0      # seconds
PROP_Q_SCALE = math.pi   # radians
PROP_N_BINS = 32         # arrival-time histogram bins
PROP_N_DIM = 8           # 7 joints + time


def proposal_features(prob: Problem, o_max: int = 32):
    """core [16], obs [o_max, 65], mask [o_max] describing one problem:
    start and goal scaled by 1/pi, the arrival range and waypoint times by
    1/60 s, each obstacle's first 16 waypoints (the last repeated) and radius."""
    core = np.zeros(PROP_CORE)
    core[:prob.d] = prob.q_start / PROP_Q_SCALE
    core[7:7 + prob.d] = prob.q_goal / PROP_Q_SCALE
    core[14] = prob.t_min / PROP_T_SCALE
    core[15] = prob.t_max / PROP_T_SCALE
    obs = np.zeros((o_max, PROP_ENC_IN))
    mask = np.zeros(o_max)
    for o in range(min(prob.n_obs, o_max)):
        n = int(prob.n_wp[o])
        for k in range(16):
            w = prob.wp[o, min(k, n - 1)]
            obs[o, 4 * k] = w[0] / PROP_T_SCALE
            obs[o, 4 * k + 1:4 * k + 4] = w[1:4]
        obs[o, 64] = prob.obs_r[o]
        mask[o] = 1.0
    return f32(core), f32(obs), mask


def proposal_targets(prob: Problem, path: np.ndarray, K: int = 16):
    """Training targets from one solution path (rows (q, t), start first):
    y [K, 8] states at K evenly spaced path indices scaled like the features
    (time in column 7, unused joints zero), ymask [K], dmask [8] (the robot's
    joints and time) and the arrival bin of the path's last time over
    [t_min, t_max] split into 32 equal bins."""
    path = np.asarray(path, dtype=np.float64)
    n = path.shape[0]
    y = np.zeros((K, PROP_N_DIM))
    ymask = np.zeros(K)
    idx = np.unique(np.round(np.linspace(0, n - 1, min(K, n))).astype(int))
    for k, i in enumerate(idx):
        y[k, :prob.d] = path[i, :prob.d] / PROP_Q_SCALE
        y[k, 7] = path[i, prob.d] / PROP_T_SCALE
        ymask[k] = 1.0
    dmask = np.zeros(PROP_N_DIM)
    dmask[:prob.d] = 1.0
    dmask[7] = 1.0
    T = float(path[-1, prob.d])
    b = int(math.floor((T - prob.t_min) / (prob.t_max - prob.t_min) * PROP_N_BINS))
    return f32(y), ymask, dmask, min(max(b, 0), PROP_N_BINS - 1)
