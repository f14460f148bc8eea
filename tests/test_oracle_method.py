"""Pins for the oracle's method steps (CPU only): counter RNG, Eq. 7 metric,
nearest node, the interval-root allocation of the paper's Fig. 2, sampling
(Eq. 6), steering, root recycling and the planner's invariants."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2609_30533_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------

def test_philox_known_answers(oracle_lib):
    from oracle.binding import philox
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# --------------------------------------------------------------------------
# Eq. 7 and nearest node
# --------------------------------------------------------------------------

def test_rho_special_cases(oracle_lib):
    prob = scenes.arm6(0)
    o = oracle_lib.Oracle(prob)
    v = prob.v_max
    rng = np.random.default_rng(0)
    for _ in range(50):
        x = np.r_[rng.uniform(-2, 2, 6), rng.uniform(0, 10)]
        u = rng.normal(size=6)
        u /= np.linalg.norm(u)
        dt = rng.uniform(0.1, 1.0)
        # on the speed cone: D = v dt, rho = D
        xr = np.r_[x[:6] + u * (v * dt * (1 - 1e-12)), x[6] + dt]
        D = np.linalg.norm(xr[:6] - x[:6])
        assert abs(o.rho(1, x, xr) - D) < 1e-9
        # zero configuration distance: rho = v |dt| / sqrt 2
        xr0 = np.r_[x[:6], x[6] + dt]
        assert abs(o.rho(1, x, xr0) - v * dt / math.sqrt(2)) < 1e-12
        # backward direction mirrors forward
        assert math.isinf(o.rho(-1, x, xr0))
        assert abs(o.rho(-1, xr0, x) - v * dt / math.sqrt(2)) < 1e-12
        # homogeneous of degree one in (dq, dt)
        xr1 = np.r_[x[:6] + 0.3 * u * v * dt, x[6] + dt]
        xr2 = np.r_[x[:6] + 0.6 * u * v * dt, x[6] + 2 * dt]
        assert abs(o.rho(1, x, xr2) - 2 * o.rho(1, x, xr1)) < 1e-12
        # outside the cone or at equal time: infinite
        assert math.isinf(o.rho(1, x, np.r_[x[:6] + u * v * dt * 1.001, x[6] + dt]))
        assert math.isinf(o.rho(1, x, np.r_[x[:6] + 0.1 * u, x[6]]))


def test_nearest_brute_force(oracle_lib):
    prob = scenes.arm6(1)
    o = oracle_lib.Oracle(prob)
    q, t, _ = scenes.synthetic_tree(prob, 300, seed=1)
    nodes = np.c_[q, t]
    rng = np.random.default_rng(2)
    v = prob.v_max
    for trial in range(60):
        xq = np.r_[rng.uniform(-math.pi, math.pi, 6), rng.uniform(0, 20)]
        sigma = 1 if trial % 2 == 0 else -1
        mask = (rng.random(300) < 0.7).astype(np.uint8)
        idx, dist, amb = o.nearest(nodes, xq, sigma=sigma, metric=0, mask=mask)
        # brute force
        best, bd = -1, math.inf
        for i in range(300):
            if not mask[i]:
                continue
            D = np.linalg.norm(nodes[i, :6] - xq[:6])
            delta = sigma * (xq[6] - nodes[i, 6])
            if delta > 0 and D <= v * delta:
                r = math.sqrt((D * D + v * v * delta * delta) / 2)
                if r < bd:
                    best, bd = i, r
        assert idx == best
        if best >= 0:
            assert abs(dist - bd) < 1e-12
        # configuration metric
        idx2, d2, _ = o.nearest(nodes, xq, metric=1)
        Ds = np.linalg.norm(nodes[:, :6] - xq[:6], axis=1)
        assert idx2 == int(np.argmin(Ds)) and abs(d2 - Ds.min()) < 1e-12


def test_nearest_ties_go_to_lowest_index(oracle_lib):
    prob = scenes.disc2d(0)
    o = oracle_lib.Oracle(prob)
    nodes = np.array([[0.5, 0.5, 1.0], [0.2, 0.2, 0.0], [0.5, 0.5, 1.0], [0.5, 0.5, 1.0]])
    idx, _, amb = o.nearest(nodes, np.array([0.5, 0.5, 2.0]), sigma=1)
    assert idx == 0 and amb
    idx, _, _ = o.nearest(nodes, np.array([0.5, 0.5, 2.0]), sigma=1, mask=np.array([0, 1, 1, 1], np.uint8))
    assert idx == 2
    idx, d, _ = o.nearest(nodes, np.array([0.5, 0.5, 0.5]), sigma=1, mask=np.array([1, 0, 1, 1], np.uint8))
    assert idx == -1 and math.isinf(d)


# --------------------------------------------------------------------------
# Interval root: the worked example of Fig. 2
# --------------------------------------------------------------------------

def _fig2():
    rows = {}
    for line in open(os.path.join(GOLDEN, "fig2_interval_root.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *vals = line.split()
        rows[k] = vals

    def iv(tok):
        a, b = tok.split(":")
        return Fraction(a), Fraction(b)
    return rows, iv


def test_fig2_worked_example(oracle_lib):
    from oracle.binding import ir_partition
    rows, iv = _fig2()
    H, N = int(rows["H"][0]), int(rows["N"][0])
    free = np.zeros(H + 1, dtype=np.uint8)
    for k in rows["free_k"]:
        free[int(k)] = 1
    for k in rows["blocked_k"]:
        assert free[int(k)] == 0
    for phase, Ubar in (("before", H), ("after", float(Fraction(rows["after.U"][0])))):
        I, pieces = ir_partition(0.0, H, Ubar, 1.0, 0, H, free, N)
        for i, tok in enumerate(rows[phase + ".uniform"]):
            lo, hi = iv(tok)
            assert abs(I[i, 0] - float(lo)) < 1e-12 and abs(I[i, 1] - float(hi)) < 1e-12
        quota = Fraction(rows[phase + ".quota"][0])
        for g in range(N):
            expect = [iv(t) for t in rows["%s.guided.%d" % (phase, g + 1)]]
            assert len(pieces[g]) == len(expect)
            for (lo, hi), p in zip(expect, pieces[g]):
                assert abs(p[0] - float(lo)) < 1e-12 and abs(p[1] - float(hi)) < 1e-12
            # exact rational check of the equal guided quota
            assert sum(hi - lo for lo, hi in expect) == quota
            assert abs(sum(p[1] - p[0] for p in pieces[g]) - float(quota)) < 1e-12
    # roots keep their group; T >= U become inactive
    U = Fraction(rows["after.U"][0])
    inactive = [Fraction(x) for x in rows["after.inactive"]]
    for tok in rows["roots"]:
        T, g = tok.split(":")
        assert (Fraction(T) >= U) == (Fraction(T) in inactive)


def test_partition_equal_division_random(oracle_lib):
    from oracle.binding import ir_partition
    rng = np.random.default_rng(4)
    for _ in range(40):
        k_lo, k_hi = 17, 17 + int(rng.integers(5, 400))
        free = (rng.random(k_hi - k_lo + 1) < rng.uniform(0.1, 0.9)).astype(np.uint8)
        dt = 0.02
        L = k_lo * dt - rng.uniform(0, dt)
        H = k_hi * dt + rng.uniform(0, dt)
        Ubar = rng.uniform(L + 0.01, H)
        N = int(rng.integers(1, 12))
        I, pieces = ir_partition(L, H, Ubar, dt, k_lo, k_hi, free, N, maxp=512)
        w = I[:, 1] - I[:, 0]
        assert np.allclose(w, (Ubar - L) / N) and abs(I[0, 0] - L) < 1e-12 and abs(I[-1, 1] - Ubar) < 1e-9
        q = [sum(p[1] - p[0] for p in pc) for pc in pieces]
        assert np.allclose(q, q[0], atol=1e-9)
        allp = sorted([tuple(p) for pc in pieces for p in pc])
        # pieces are disjoint, inside [L, Ubar), each inside a free check's window
        for a, b in zip(allp, allp[1:]):
            assert a[1] <= b[0] + 1e-12
        for lo, hi in allp:
            assert lo >= L - 1e-12 and hi <= Ubar + 1e-12
            mid = 0.5 * (lo + hi)
            k = int(round(mid / dt))
            assert free[k - k_lo] == 1 or free[min(k + 1, k_hi) - k_lo] or free[max(k - 1, k_lo) - k_lo]
        # total guided duration = free windows clipped to [L, Ubar)
        tot = 0.0
        for k in range(k_lo, k_hi + 1):
            if free[k - k_lo]:
                tot += max(0.0, min(k * dt + dt / 2, H, Ubar) - max(k * dt - dt / 2, L))
        assert abs(sum(q) - tot) < 1e-9


# --------------------------------------------------------------------------
# Sampling (Eq. 6) and steering
# --------------------------------------------------------------------------

def test_sampling_bounds_and_mixture(oracle_lib):
    prob = scenes.disc2d(0)
    prob.params.batch = 20000
    pl = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    inf = pl.info()
    s = pl.sample(0)
    v = prob.v_max
    ok = (s["flags"] & 1) == 0
    assert ok.sum() > 1000
    # group uniform over {0..N-1}
    counts = np.bincount(s["grp"], minlength=4)
    assert np.all(np.abs(counts / 20000 - 0.25) < 0.02)
    # q_r inside the box; Eq. 6 bounds on t_r
    q = s["qr"].T
    assert np.all(q >= prob.q_lo) and np.all(q <= prob.q_hi)
    lo = np.linalg.norm(q - prob.q_start, axis=1) / v
    hi = s["T"] - np.linalg.norm(q - prob.q_goal, axis=1) / v
    assert np.all(s["tr"][ok] >= lo[ok] - 1e-12) and np.all(s["tr"][ok] <= hi[ok] + 1e-12)
    # every rejected-for-empty-interval sample really had hi < lo, or a blocked root
    rej = ~ok
    for i in np.where(rej)[0][:200]:
        root_ok, _ = o.state_valid(np.r_[prob.q_goal, s["T"][i]])
        assert (hi[i] < lo[i]) or not root_ok
    # T lies in [L, Ubar)
    assert np.all(s["T"] >= inf["L"] - 1e-12) and np.all(s["T"] < inf["H"])
    # direction alternates with worker index
    assert np.array_equal(s["dir"], (np.arange(20000) % 2).astype(np.int8))
    # backward samples in groups without trees always use a virtual root
    bwd = (s["dir"] == 1) & ok
    assert np.all((s["flags"][bwd] & 2) != 0)


def test_root_time_distribution_chi2(oracle_lib):
    """T follows the mixture: p_guided on the group's guided portions, the rest
    uniform on I_i (chi-square over the group's interval)."""
    prob = scenes.disc2d(2)
    prob.params.batch = 200000
    pl = oracle_lib.Planner(prob)
    s = pl.sample(0)
    I, pieces = pl.partition()
    pg = prob.params.p_guided
    for g in range(prob.params.n_groups):
        Tg = s["T"][s["grp"] == g]
        lo, hi = I[g]
        nb = 40
        edges = np.linspace(min(lo, min([p[0] for p in pieces[g]], default=lo)),
                            max(hi, max([p[1] for p in pieces[g]], default=hi)), nb + 1)
        obs, _ = np.histogram(Tg, bins=edges)
        Gi = sum(p[1] - p[0] for p in pieces[g])
        expect = np.zeros(nb)
        for b in range(nb):
            a, c = edges[b], edges[b + 1]
            u = max(0.0, min(c, hi) - max(a, lo)) / (hi - lo)
            gd = sum(max(0.0, min(c, p[1]) - max(a, p[0])) for p in pieces[g]) / Gi if Gi > 0 else 0.0
            expect[b] = len(Tg) * ((pg * gd + (1 - pg) * u) if Gi > 0 else u)
        m = expect > 5
        chi2 = ((obs[m] - expect[m]) ** 2 / expect[m]).sum()
        dof = m.sum() - 1
        assert chi2 < dof + 5 * math.sqrt(2 * dof), (g, chi2, dof)
        assert obs[~m].sum() <= expect[~m].sum() + 5 * math.sqrt(expect[~m].sum() + 1) + 5


def test_steer_invariants_interval_root(oracle_lib):
    prob = scenes.arm6(5)
    prob.params.batch = 512
    pl = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    snap0 = pl.export()
    s = pl.sample(0)
    out = pl.extend(s)
    v = prob.v_max
    eta = prob.params.eta
    adv = np.where(out["status"] == 2)[0]
    assert len(adv) > 10
    snap = pl.export()
    for i in adv:
        xnew = out["xnew"][:, i]
        par = out["parent"][i]
        xn = snap["x"][par]
        sigma = 1 if s["dir"][i] == 0 else -1
        xr = np.r_[s["qr"][:, i], s["tr"][i]]
        # same fraction in q and t: rho(x_n, x_new) = min(eta, rho(x_n, x_r))
        assert abs(o.rho(sigma, xn, xnew) - min(eta, o.rho(sigma, xn, xr))) < 1e-9
        D = np.linalg.norm(xnew[:6] - xn[:6])
        assert sigma * (xnew[6] - xn[6]) > 0 and D <= v * abs(xnew[6] - xn[6]) * (1 + 1e-12)
    del snap0


def test_root_recycling_invariants(oracle_lib):
    prob = scenes.arm7rr(1, n_obs=8)
    prob.params.batch = 512
    prob.params.cap_bwd = 1 << 12
    pl = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    inf = pl.info()
    T0, act0, gen0, k0 = pl.slots()
    Lgrid = math.ceil(inf["L"] / prob.params.dt) * prob.params.dt
    for s in range(prob.params.n_groups):
        if act0[s]:
            assert T0[s] >= Lgrid - 1e-12 and T0[s] < prob.t_max
            assert abs(T0[s] - k0[s] * prob.params.dt) < 1e-12
            assert o.state_valid(np.r_[prob.q_goal, T0[s]])[0]
    prevU = math.inf
    prev_gen = gen0.copy()
    for it in range(30):
        s = pl.sample(it)
        # backward workers go round-robin over the active slots
        T, act, gen, _ = pl.slots()
        active = np.where(act)[0]
        bwd = np.where((s["dir"] == 1) & ((s["flags"] & 1) == 0))[0]
        if len(active):
            assert np.array_equal(s["grp"][bwd], active[(bwd // 2) % len(active)])
        snap_before = pl.export()
        out = pl.extend(s)
        inf = pl.info()
        T, act, gen, kk = pl.slots()
        assert np.all(gen >= prev_gen)
        if inf["U"] < prevU:
            U = inf["U"]
            assert np.all(T[act == 1] < U)
            for sl in np.where(gen > prev_gen)[0]:
                assert Lgrid - 1e-12 <= T[sl] < U and o.state_valid(np.r_[prob.q_goal, T[sl]])[0]
                assert pl.counts()[1 + sl] == 1
            # the forward tree is untouched by recycling
            c = pl.counts()
            after = pl.export()
            assert np.array_equal(after["x"][:snap_before["counts"][0]], snap_before["x"][:snap_before["counts"][0]])
            del c
        prevU = inf["U"]
        prev_gen = gen.copy()
        del out


def test_no_recycling_keeps_the_initial_roots(oracle_lib):
    """The allocation ablation of the evaluation: the same initial roots as
    recycling, deactivation at a drop of U, never a replacement; until the
    first drop of U both runs are identical."""
    prob = scenes.arm7rr(1, n_obs=8)
    prob.params.batch = 512
    prob.params.cap_bwd = 1 << 12
    rec = oracle_lib.Planner(prob)
    prob2 = scenes.arm7rr(1, n_obs=8)
    prob2.params.batch = 512
    prob2.params.cap_bwd = 1 << 12
    prob2.params.no_recycling = 1
    fix = oracle_lib.Planner(prob2)
    T0, act0, gen0, k0 = fix.slots()
    Tr, actr, genr, kr = rec.slots()
    assert np.array_equal(T0, Tr) and np.array_equal(act0, actr) and np.array_equal(k0, kr)
    prevU, drops, same = math.inf, 0, True
    for it in range(40):
        s1, s2 = rec.sample(it), fix.sample(it)
        if same:
            assert np.array_equal(s1["qr"], s2["qr"]) and np.array_equal(s1["grp"], s2["grp"])
        rec.extend(s1)
        fix.extend(s2)
        T, act, gen, kk = fix.slots()
        assert np.array_equal(gen, gen0) and np.array_equal(kk, k0)
        assert np.array_equal(T[act == 1], T0[act == 1])
        assert np.all(act <= act0)
        U = fix.info()["U"]
        if U < prevU:
            drops += 1
            assert np.all(T[act == 1] < U)
            assert np.all(act[(T0 >= U) & (act0 == 1)] == 0)
        if drops > 0:
            same = False  # the allocations differ from the first drop of U on
        prevU = U
    assert drops >= 1


# --------------------------------------------------------------------------
# Planner invariants and closed-form arrival cases
# --------------------------------------------------------------------------

def _tree_invariants(prob, snap, counts, N, cap_f, cap_b):
    v = prob.v_max
    d = prob.d
    x, par = snap["x"], snap["parent"]
    for pool in range(1 + N):
        base = 0 if pool == 0 else cap_f + (pool - 1) * cap_b
        for i in range(base, base + counts[pool]):
            p = par[i]
            if p < 0:
                continue
            dtp = x[i, d] - x[p, d]
            if pool == 0:
                assert dtp > 0            # forward parents are earlier
            else:
                assert dtp < 0            # backward parents are later
            D = np.linalg.norm(x[i, :d] - x[p, :d])
            assert D <= v * abs(dtp) * (1 + 1e-9) + 1e-12
            assert abs(snap["cost"][i] - snap["cost"][p] - D) < 1e-9


@pytest.mark.parametrize("variant", [0, 1])
def test_planner_paths_valid_and_tree_invariants(oracle_lib, variant):
    for seed in range(3):
        prob = scenes.disc2d(seed)
        prob.params.variant = variant
        prob.params.n_groups = 4 if variant == 0 else 8
        pl = oracle_lib.Planner(prob)
        o = oracle_lib.Oracle(prob)
        r = pl.run(60)
        inf = pl.info()
        snap = pl.export()
        _tree_invariants(prob, snap, pl.counts(), prob.params.n_groups, prob.params.cap_fwd, prob.params.cap_bwd)
        if r == 0:
            path = pl.path()
            ok, msg = o.validate_path(path, inf["U"], inf["C"])
            assert ok, msg
            assert inf["U"] >= inf["L"] - 1e-12


def test_obstacle_free_arrival_tends_to_lower_bound(oracle_lib):
    prob = scenes.disc2d(3)
    prob.wp[:, :, 1:3] = 50.0        # move every obstacle far away
    prob.t_min = 0.0
    pl = oracle_lib.Planner(prob)
    pl.run(400)
    inf = pl.info()
    Lg = np.linalg.norm(prob.q_start - prob.q_goal) / prob.v_max
    assert abs(inf["L"] - Lg) < 1e-12
    assert Lg <= inf["U"] <= Lg + 0.05


def test_goal_blocked_until_time_gives_arrival_after_unblock(oracle_lib):
    """An obstacle parked on the goal until t = 4 s and then gone: no path can
    arrive earlier, and the planner arrives shortly after."""
    prob = scenes.disc2d(4)
    g = prob.q_goal
    far = [40.0, 40.0]
    prob.n_wp = np.full(prob.n_obs, 2, dtype=np.int32)
    wp = np.zeros((prob.n_obs, 4, 4))
    wp[:, :, 1:3] = far
    wp[:, 0, 0], wp[:, 1, 0] = 0.0, 10.0
    prob.wp = wp[:, :2].copy()
    prob.n_wp[0] = 4
    w0 = np.array([[0.0, g[0], g[1], 0.0], [4.0, g[0], g[1], 0.0], [4.001, 40.0, 40.0, 0.0], [10.0, 40.0, 40.0, 0.0]])
    prob.wp = np.zeros((prob.n_obs, 4, 4))
    prob.wp[:, :2] = wp[:, :2]
    prob.wp[0] = w0
    prob.t_min = 0.0
    pl = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    pl.run(300)
    inf = pl.info()
    assert inf["U"] >= 4.0
    assert inf["U"] <= 4.2
    ok, msg = o.validate_path(pl.path(), inf["U"], inf["C"])
    assert ok, msg


def test_trivial_case(oracle_lib):
    prob = scenes.disc2d(0)
    prob.q_goal = prob.q_start.copy()
    prob.t_min = 0.0
    prob.wp[:, :, 1:3] = 50.0
    pl = oracle_lib.Planner(prob)
    assert pl.run(5) == 2
    prob.t_min = 2.0     # arrival at time 0 not allowed: plan normally
    pl2 = oracle_lib.Planner(prob)
    assert pl2.run(50) == 0 and pl2.info()["U"] >= 2.0
