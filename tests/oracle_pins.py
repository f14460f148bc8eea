"""Pins of the FP64 oracle against what the paper and plain mathematics fix.

Each pin is a plain function that raises AssertionError when the oracle
disagrees with the definition it follows.  They are collected as CPU tests by
``test_oracle_pins.py`` and re-run by ``test_oracle_mutants.py`` against
copies of the oracle with one plausible mistake planted, where each must
fail.  The docstring of every pin names the mistakes it is meant to catch.

The brute-force references below are written from the definitions (Eq. 7,
Eq. 8, Sec. IV-B bridge ranking, the capacity reading of the batch commit),
not from the oracle's code, and share nothing with it.
"""
import math
import os

import numpy as np

from paper_2609_30533_amd import scenes

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FLAG_SKIP, FLAG_USE_NEW, FLAG_LEARNED = 1, 2, 4
ST_ADVANCED, ST_DROPPED = 2, 3


# --------------------------------------------------------------------------
# bridge ranking (Sec. IV-B: admissible candidates ranked by arrival time,
# then by the space-time distance; Alg. 1 tests only the best-ranked one)
# --------------------------------------------------------------------------

def _rho_def(v, sigma, x, y, d):
    """Eq. 7 from x to y in direction sigma: infinite unless the time step
    sigma (t_y - t_x) is positive and the configuration distance fits the
    speed limit over it."""
    D = float(np.linalg.norm(np.asarray(y[:d]) - np.asarray(x[:d])))
    delta = sigma * (y[d] - x[d])
    if not (delta > 0 and D <= v * delta):
        return math.inf
    return math.sqrt((D * D + (v * (y[d] - x[d])) ** 2) / 2.0)


def _random_forest(prob, rng, n_fwd, trees_per_pool, nodes_per_tree):
    """A forward tree and a few backward trees per pool, laid out in the
    global numbering (pool 0 at 0, pool 1+i at cap_fwd + i cap_bwd).  Node
    times respect the tree directions; costs are not used by the ranking."""
    P = prob.params
    d = prob.d
    N = P.n_groups
    total = P.cap_fwd + N * P.cap_bwd
    x = np.zeros((total, d + 1))
    parent = np.full(total, -1, dtype=np.int32)
    rootT = np.zeros(total)
    cost = np.zeros(total)
    counts = np.zeros(1 + N, dtype=np.int64)
    H = prob.t_max
    for i in range(n_fwd):
        x[i, :d] = rng.uniform(prob.q_lo, prob.q_hi)
        x[i, d] = 0.0 if i == 0 else rng.uniform(0.0, 0.6 * H)
        parent[i] = -1 if i == 0 else 0
    counts[0] = n_fwd
    for g in range(N):
        base = P.cap_fwd + g * P.cap_bwd
        k = 0
        for _ in range(trees_per_pool):
            T = rng.uniform(0.4 * H, H)
            r = base + k
            x[r, :d] = prob.q_goal
            x[r, d] = T
            rootT[r] = T
            k += 1
            for _ in range(nodes_per_tree):
                i = base + k
                x[i, :d] = rng.uniform(prob.q_lo, prob.q_hi)
                x[i, d] = rng.uniform(0.2 * H, T)
                parent[i] = r
                rootT[i] = T
                k += 1
        counts[1 + g] = k
    return counts, x, parent, cost, rootT


def pin_bridge_ranking(oracle):
    """Brute force over random forests: the chosen bridge is the admissible
    candidate of least (arrival, rho, index), arrival being the candidate
    tree's root time for a forward new node and the new node's own root time
    for a backward one; backward trees rooted at or after U are not
    candidates.

    Catches: ranking by rho before arrival; taking the arrival from the new
    node's tree for forward nodes; keeping trees rooted at T >= U; searching
    the same side instead of the opposite one."""
    rng = np.random.default_rng(11)
    prob = scenes.disc2d(5)
    P = prob.params
    P.n_groups, P.cap_fwd, P.cap_bwd = 3, 64, 48
    d, v = prob.d, prob.v_max
    pl = oracle.Planner(prob)
    n_checked = n_arrival_matters = n_u_matters = 0
    for trial in range(12):
        counts, x, parent, cost, rootT = _random_forest(prob, rng, 40, 3, 12)
        roots = sorted(rootT[(parent < 0) & (rootT > 0)])
        U = 0.5 * (roots[len(roots) // 2] + roots[len(roots) // 2 + 1])  # about half the trees inactive
        pl.import_state(counts, x, parent, cost, rootT, U, 5.0, -1, -1, 0)
        fwd = list(range(int(counts[0])))
        bwd = [P.cap_fwd + g * P.cap_bwd + k for g in range(P.n_groups) for k in range(int(counts[1 + g]))]
        for q in range(40):
            sigma = 1 if q % 2 == 0 else -1
            xq = np.r_[rng.uniform(prob.q_lo, prob.q_hi), rng.uniform(0.1 * prob.t_max, 0.97 * prob.t_max)]
            x_root = rng.uniform(0.4 * prob.t_max, prob.t_max)
            cands = bwd if sigma > 0 else fwd
            keys, keys_rho, keys_all = [], [], []
            for i in cands:
                r = _rho_def(v, sigma, xq, x[i], d)
                if math.isinf(r):
                    continue
                arr = rootT[i] if sigma > 0 else x_root
                keys_all.append((arr, r, i))
                if sigma > 0 and not rootT[i] < U:
                    continue
                keys.append((arr, r, i))
                keys_rho.append((r, i))
            expect = min(keys)[2] if keys else -1
            b, arr, amb = pl.bridge(sigma, xq, x_root)
            if amb:
                continue
            assert b == expect, (trial, q, sigma, b, expect)
            if keys:
                assert abs(arr - min(keys)[0]) <= 1e-12
                n_arrival_matters += int(min(keys_rho)[1] != expect)
            # trees rooted at T >= U rank after every active one; they decide
            # only when no active candidate is admissible
            n_u_matters += int(bool(keys_all) and min(keys_all)[2] != expect)
            n_checked += 1
    # the random forests do separate the alternatives the docstring names
    assert n_checked >= 300 and n_arrival_matters >= 20 and n_u_matters >= 10, (
        n_checked, n_arrival_matters, n_u_matters)


# --------------------------------------------------------------------------
# maximum-speed extension of root recycling (Sec. V, Eq. 8)
# --------------------------------------------------------------------------

def pin_eq8_max_speed_step(oracle):
    """Every advanced recycling worker moves from its nearest node q_n (by
    configuration distance) toward q_r by min(1, eta / D(q_n, q_r)) of the
    way, and is timed at maximum speed: D(q_n, q_new) = v_max |t_new - t_n|
    exactly, with the time moving in the worker's direction.

    Catches: timing the step with the untruncated distance D(q_n, q_r); not
    capping the step at eta; a wrong time direction for backward workers;
    choosing the parent by Eq. 7 instead of the configuration distance."""
    prob = scenes.arm7rr(1, n_obs=8)
    P = prob.params
    P.batch, P.n_groups, P.cap_bwd = 512, 16, 1 << 12
    d, v, eta = prob.d, prob.v_max, P.eta
    pl = oracle.Planner(prob)
    n_adv = n_capped = 0
    for it in range(8):
        snap = pl.export()
        s = pl.sample(it)
        out = pl.extend(s)
        for w in np.where(out["status"] == ST_ADVANCED)[0]:
            par = int(out["parent"][w])
            xn = snap["x"][par]
            xnew = out["xnew"][:, w]
            qr = s["qr"][:, w]
            sigma = 1 if s["dir"][w] == 0 else -1
            # the parent is the nearest node of the worker's tree by configuration distance
            pool = 0 if sigma > 0 else 1 + int(s["grp"][w])
            base = 0 if pool == 0 else P.cap_fwd + (pool - 1) * P.cap_bwd
            nodes = snap["x"][base:base + int(snap["counts"][pool]), :d]
            Dall = np.linalg.norm(nodes - qr, axis=1)
            assert par - base == int(np.argmin(Dall)), (it, w)
            Dr = float(np.linalg.norm(qr - xn[:d]))
            f = min(1.0, eta / Dr)
            np.testing.assert_allclose(xnew[:d], xn[:d] + f * (qr - xn[:d]), rtol=0, atol=1e-12)
            D = float(np.linalg.norm(xnew[:d] - xn[:d]))
            assert D <= eta * (1 + 1e-12) + 1e-15
            assert abs(D - v * abs(xnew[d] - xn[d])) <= 1e-12 * max(1.0, D)
            assert sigma * (xnew[d] - xn[d]) > 0
            n_adv += 1
            n_capped += int(f < 1.0)
    assert n_adv >= 50 and n_capped >= 20, (n_adv, n_capped)


# --------------------------------------------------------------------------
# path validator (the re-check every returned path goes through)
# --------------------------------------------------------------------------

def _open_field(seed=6):
    """A disc problem whose obstacles are parked far away."""
    prob = scenes.disc2d(seed)
    prob.wp[:, :, 1:3] = 50.0
    return prob


def _straight_path(prob, U, n=5):
    """(q_s, 0) ... (q_g, U) along the straight segment at constant speed."""
    s = np.linspace(0.0, 1.0, n)
    q = prob.q_start[None, :] + s[:, None] * (prob.q_goal - prob.q_start)[None, :]
    return np.c_[q, s * U], float(np.linalg.norm(prob.q_goal - prob.q_start))


def pin_validator_rejections(oracle):
    """The validator accepts a straight constant-speed path in an empty
    field and rejects, each with its own reason, a path whose time does not
    increase, that exceeds the speed limit, that crosses an obstacle, that
    does not start at (q_s, 0), that does not end at (q_g, U), whose U lies
    outside the arrival range, or whose length differs from C.

    Catches: a missing or inverted check of any of these conditions (a
    removed time test would report the speed test instead; a removed
    collision test would accept the blocked path)."""
    prob = _open_field()
    o = oracle.Oracle(prob)
    d = prob.d
    L = max(np.linalg.norm(prob.q_goal - prob.q_start) / prob.v_max, prob.t_min)
    U = L + 1.0
    path, C = _straight_path(prob, U)
    ok, msg = o.validate_path(path, U, C)
    assert ok, msg

    def rejects(p, U_, C_, reason, prob_=None):
        ok_, msg_ = (oracle.Oracle(prob_) if prob_ is not None else o).validate_path(p, U_, C_)
        assert not ok_ and reason in msg_, (reason, msg_)

    bad = path.copy()
    bad[2, d] = bad[1, d]                         # equal times
    rejects(bad, U, C, "time not increasing")
    bad = path.copy()
    bad[2, d], bad[1, d] = bad[1, d], bad[2, d]   # time runs backwards
    rejects(bad, U, C, "time not increasing")
    bad = path.copy()
    bad[2, d] = bad[1, d] + 1e-3                  # one segment far above the speed limit
    rejects(bad, U, C, "speed bound")
    bad = path.copy()
    bad[0, :d] += 0.01
    rejects(bad, U, C, "first state is not q_s")
    bad = path.copy()
    bad[0, d] = 1e-3
    rejects(bad, U, C, "first state time")
    bad = path.copy()
    bad[-1, :d] += 0.01
    rejects(bad, U, C, "last state is not q_g")
    rejects(path, U + 0.1, C, "!= U")
    rejects(path, U, C * 1.01, "length")
    # arrival outside the range: the same path timed to end before t_min,
    # and after t_max
    early = path.copy()
    early[:, d] *= (0.9 * prob.t_min) / U
    prob_fast = _open_field()
    prob_fast.v_max = 100.0
    rejects(early, early[-1, d], C, "outside", prob_fast)
    late = path.copy()
    late[:, d] *= (prob.t_max + 1.0) / U
    rejects(late, late[-1, d], C, "outside")
    # an obstacle parked on the middle of the segment for the whole horizon
    prob_b = _open_field()
    mid = 0.5 * (prob_b.q_start + prob_b.q_goal)
    prob_b.wp[0, :, 1:3] = mid
    rejects(path, U, C, "collides", prob_b)


# --------------------------------------------------------------------------
# capacity (reading: atomic slot claims in worker order; a suffix is dropped)
# --------------------------------------------------------------------------

def pin_capacity_suffix(oracle):
    """With tiny pools, the workers of each pool that advanced claim
    consecutive slots in worker order (two for a backward worker whose
    virtual root is materialised, one otherwise); a worker is inserted iff
    its claim, counting the claims of every earlier worker of the pool,
    dropped or not, ends within the pool's capacity; the pool count grows by
    the inserted claims only.

    Catches: a claim counter that does not advance on a drop (a later
    one-slot worker then fits after a dropped two-slot one); counting a
    virtual-root insert as one slot; dropping whole batches instead of a
    suffix."""
    n_gap_cases = n_drops = 0
    for seed in (1, 2, 3):
        prob = scenes.disc2d(seed)
        P = prob.params
        P.batch, P.n_groups, P.cap_fwd, P.cap_bwd, P.p_new = 256, 4, 60, 9, 0.5
        pl = oracle.Planner(prob)
        for it in range(6):
            c0 = pl.counts().copy()
            s = pl.sample(it)
            out = pl.extend(s)
            c1 = pl.counts()
            st = out["status"]
            drops_before = n_drops
            for pool in range(1 + P.n_groups):
                cap = P.cap_fwd if pool == 0 else P.cap_bwd
                claim = int(c0[pool])
                inserted = 0
                for w in range(P.batch):
                    if st[w] not in (ST_ADVANCED, ST_DROPPED):
                        continue
                    wpool = 0 if s["dir"][w] == 0 else 1 + int(s["grp"][w])
                    if wpool != pool:
                        continue
                    need = 2 if (s["dir"][w] == 1 and (s["flags"][w] & FLAG_USE_NEW)) else 1
                    claim += need
                    if claim <= cap:
                        assert st[w] == ST_ADVANCED, (seed, it, pool, w)
                        inserted += need
                    else:
                        assert st[w] == ST_DROPPED, (seed, it, pool, w)
                        n_drops += 1
                        # dropped although it would fit on its own behind the
                        # inserted workers: only the claim rule drops it
                        n_gap_cases += int(c0[pool] + inserted + need <= cap)
                assert int(c1[pool]) == int(c0[pool]) + inserted, (seed, it, pool)
            if n_drops > drops_before:
                assert pl.info()["overflow"] == 1.0
    assert n_drops >= 20 and n_gap_cases >= 1, (n_drops, n_gap_cases)


# --------------------------------------------------------------------------
# learned draw (readings 16-17 of the added proposal): a diagonal Gaussian
# mixture over the normalised state (q / pi, t / 60), an arrival histogram
# --------------------------------------------------------------------------

def _proposal_output(n_comp=8):
    """A network output z[168] with well-separated components (means along
    joint 0 at -0.7, -0.5, ..., 0.7, standard deviation 0.02 there) and
    distinct weights and arrival-histogram logits."""
    z = np.zeros(168)
    z[:8] = np.linspace(-1.0, 1.0, 8)                    # mixture logits
    mu = np.zeros((8, 8))
    lsd = np.zeros((8, 8))
    for c in range(n_comp):
        mu[c, 0] = -0.7 + 0.2 * c
        lsd[c, 0] = math.log(0.02)
        for j in range(1, 7):
            mu[c, j] = 0.1 * (j - 3) + 0.02 * c
            lsd[c, j] = math.log(0.05 + 0.01 * j + 0.005 * c)
        mu[c, 7] = 0.1 + 0.01 * c
        lsd[c, 7] = math.log(0.01)
    z[8:72] = mu.ravel()
    z[72:136] = lsd.ravel()
    z[136:168] = np.sin(np.arange(32)) * 1.5              # histogram logits
    return z, mu, np.exp(lsd)


def _softmax(a):
    e = np.exp(a - np.max(a))
    return e / e.sum()


def _chi2_ok(obs, p, n):
    exp_ = p * n
    m = exp_ > 5
    chi2 = float(((obs[m] - exp_[m]) ** 2 / exp_[m]).sum())
    dof = int(m.sum()) - 1
    return chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def pin_learned_draw_moments(oracle):
    """Draws of the learned proposal follow the installed mixture: the
    component frequencies match the softmax weights (chi-square), each
    component's joint draws have mean pi mu and standard deviation pi sigma
    with sigma = exp(log sd) (five standard errors), the arrival-histogram
    bins of the root time T match the softmax of the histogram logits, and
    the fraction of learned draws is the mixing probability.

    Catches: using the log standard deviation as the standard deviation;
    dropping the pi scaling of the configuration; a Box-Muller angle over
    half a turn (one-signed variates); an off-by-one in the component or
    bin choice; a mixing decision against the wrong probability."""
    z, mu, sd = _proposal_output()
    w = _softmax(z[:8])
    # recycling: only q comes from the network
    prob = scenes.arm7rr(4, n_obs=8)
    P = prob.params
    P.n_groups, P.cap_bwd = 8, 1 << 10
    n = 1 << 16
    pl = oracle.Planner(prob)
    pl.set_proposal(z, 1.0)
    s = pl.sample(0, n)
    learned = (s["flags"] & FLAG_LEARNED) != 0
    assert learned.all()
    qn = s["qr"] / math.pi
    comp = np.rint((qn[0] + 0.7) / 0.2).astype(int)
    assert comp.min() >= 0 and comp.max() <= 7
    assert np.all(np.abs(qn[0] - (-0.7 + 0.2 * comp)) < 0.1)
    counts = np.bincount(comp, minlength=8)
    ok, info = _chi2_ok(counts, w, n)
    assert ok, info
    for c in range(8):
        sel = qn[:, comp == c]
        m = sel.shape[1]
        for j in range(prob.d):
            se = sd[c, j] / math.sqrt(m)
            assert abs(sel[j].mean() - mu[c, j]) < 5 * se, (c, j, sel[j].mean(), mu[c, j])
            sd_hat = sel[j].std(ddof=1)
            assert abs(sd_hat - sd[c, j]) < 5 * sd[c, j] / math.sqrt(2 * (m - 1)), (c, j, sd_hat, sd[c, j])
    # interval root: T from the arrival histogram over [t_min, t_max]
    prob2 = scenes.disc2d(4)
    prob2.params.n_groups = 4
    pl2 = oracle.Planner(prob2)
    pl2.set_proposal(z, 1.0)
    s2 = pl2.sample(0, n)
    width = (prob2.t_max - prob2.t_min) / 32.0
    b = np.floor((s2["T"] - prob2.t_min) / width).astype(int)
    assert b.min() >= 0 and b.max() <= 31
    ok, info = _chi2_ok(np.bincount(b, minlength=32), _softmax(z[136:168]), n)
    assert ok, info
    # mixing probability
    pl3 = oracle.Planner(prob2)
    pl3.set_proposal(z, 0.3)
    s3 = pl3.sample(0, n)
    frac = float(((s3["flags"] & FLAG_LEARNED) != 0).mean())
    assert abs(frac - 0.3) < 5 * math.sqrt(0.3 * 0.7 / n), frac


def _rr_worked():
    rows = {}
    for line in open(os.path.join(GOLDEN, "rr_worked_example.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, rest = line.split(None, 1)
            rows[k] = rest
    return rows


def pin_recycling_worked_example(oracle):
    """Root recycling on a hand-worked scene (tests/golden/rr_worked_example.txt,
    Sec. V / Alg. 3, readings 12-13): the initial slot roots and the roots
    after a drop of U equal the values derived by hand.  Catches: strata over
    the wrong index range (k dt <= H, or [L, H) after the drop instead of
    k dt < U), a stratum's first grid time taken whether free or not,
    occupied strata not skipped, donors taken with T >= U or in the wrong
    order, a donor consumed by a stratum without a free index, the
    generation not advanced."""
    prob, rows = rr_worked_problem()
    pl = oracle.Planner(prob)
    ints = lambda key: np.array([int(v) for v in rows[key].split()])
    flts = lambda key: np.array([float(v) for v in rows[key].split()])
    T, act, gen, k = pl.slots()
    assert np.array_equal(k, ints("init.k")), k
    assert np.allclose(T, flts("init.T"), atol=1e-12), T
    assert np.array_equal(act, ints("init.active")), act
    pl.recycle(float(rows["U"]))
    T, act, gen, k = pl.slots()
    assert np.array_equal(k, ints("after.k")), k
    assert np.allclose(T, flts("after.T"), atol=1e-12), T
    assert np.array_equal(act, ints("after.active")), act
    assert np.array_equal(gen, ints("after.gen")), gen


def rr_worked_problem():
    """The scene of tests/golden/rr_worked_example.txt and its rows."""
    rows = _rr_worked()
    wp = np.array([[float(v) for v in seg.split()] for seg in rows["wp"].split("|")])
    prob = scenes.Problem(
        name="rr-worked", d=2, kind=scenes.KIND_TRANSLATE, dh=np.zeros((2, 4)),
        sphere_link=np.zeros(1, dtype=np.int32), sphere=scenes.f32(np.array([[0.0, 0.0, 0.0, 0.05]])),
        q_lo=scenes.f32(np.zeros(2)), q_hi=scenes.f32(np.ones(2)), q_start=scenes.f32([0.3, 0.5]),
        q_goal=scenes.f32([0.8, 0.5]), t_min=scenes.f32(2.0), t_max=scenes.f32(10.0), v_max=scenes.f32(1.0),
        n_wp=np.array([len(wp)], dtype=np.int32), wp=scenes.f32(wp[None]), obs_r=scenes.f32([0.08]),
        params=scenes.Params(variant=scenes.VARIANT_RR, n_groups=4, batch=64, eta=0.1, h=0.01, dt=0.02,
                             cap_fwd=1 << 10, cap_bwd=1 << 8, seed=1),
        seed=0)
    return prob, rows



PINS = {
    "recycling_worked_example": pin_recycling_worked_example,
    "bridge_ranking": pin_bridge_ranking,
    "eq8_max_speed_step": pin_eq8_max_speed_step,
    "validator_rejections": pin_validator_rejections,
    "capacity_suffix": pin_capacity_suffix,
    "learned_draw_moments": pin_learned_draw_moments,
}
