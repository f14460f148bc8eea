"""Parity of the sampling, extend and planning entry points with the oracle.

The extend batch is compared iteration by iteration on identical inputs: the
device state is exported after every batch, rounded to FP32 and imported into
the oracle (resynchronised lockstep), the device draws the samples and both
sides run Alg. 1 on them.  Decisions must agree exactly except where the
oracle flags a numerically fragile choice (near-tie or near speed cone,
clearance within 1e-4); continuous results agree within a relative 1e-5.
Every planned path is re-validated by the oracle."""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu

MARGIN = 1e-4


def _small(prob, batch, cap_f=1 << 14, cap_b=1 << 11, groups=None):
    prob.params.batch = batch
    prob.params.cap_fwd = cap_f
    prob.params.cap_bwd = cap_b
    if groups:
        prob.params.n_groups = groups
    return prob


def _c3_parked(seed):
    """The recycling workload at its full shape (7-DOF arm, 60 spheres, 32
    moving spheres x 16 waypoints, 64 slots, B = 8192, pools 2^18 / 2^14) with
    obstacles 8..31 moved 3 m away along y: every obstacle is still
    interpolated and tested, but the problem is solvable before the forward
    pool fills (about 64 iterations of 4096 forward workers)."""
    prob = scenes.arm7rr(seed)
    prob.wp[8:, :, 1] += 3.0
    return prob


def _no_recycling(prob):
    prob.params.no_recycling = 1
    return prob


def _tiny_pools(prob, p_new=0.5):
    """Pools of a few dozen nodes, so that inserts are dropped within a few
    iterations; a raised p_new gives many two-slot (virtual-root) claims."""
    prob.params.cap_fwd = 60
    prob.params.cap_bwd = 9
    prob.params.p_new = p_new
    return prob


def _to_np(s):
    return {k: v.cpu().numpy() for k, v in s.items()}


def _resync(gp, op, prob):
    """Load the device state into the oracle planner."""
    st = gp.export()
    inf = gp.info()
    slots = gp.slots() if prob.params.variant == 1 else None
    op.import_state(st["counts"], st["x"].astype(np.float64), st["parent"], st["cost"].astype(np.float64),
                    st["rootT"].astype(np.float64), inf["U"], inf["C"], inf["inc_fwd"], inf["inc_bwd"], inf["iter"],
                    slots)
    return st


PROBS = [
    ("disc2d-ir", lambda: _small(scenes.disc2d(1), 512)),
    ("arm6-ir", lambda: _small(scenes.arm6(2), 1024, groups=8)),
    ("disc2d-rr", lambda: _small(scenes.disc2d(2, params=scenes.Params(variant=1, n_groups=8)), 512)),
    ("arm7-rr", lambda: _small(scenes.arm7rr(2, n_obs=16), 1024, groups=16)),
    ("arm7-norecycle", lambda: _no_recycling(_small(scenes.arm7rr(2, n_obs=16), 1024, groups=16))),
    # the start configuration is grazed by an obstacle at t ~ 0.43 s: most
    # forward edges pass within 1e-4 m of contact (exempt decisions)
    ("arm6-ir-grazing", lambda: _small(scenes.arm6(1), 1024, groups=8)),
    # a batch that fills no launch shape evenly (ragged blocks and tiles)
    ("arm6-ir-ragged", lambda: _small(scenes.arm6(2), 1000 + 7, groups=8)),
    # self-collision and fixed boxes switched on
    ("arm6-static-ir", lambda: _small(scenes.arm6static(8), 1024, groups=8)),
    ("arm7-static-rr", lambda: _small(scenes.with_static(scenes.arm7rr(30, n_obs=8)), 1024, groups=16)),
    # pools that fill up: dropped inserts (a suffix per pool), two-slot
    # virtual-root claims at the boundary
    ("disc2d-capacity", lambda: _tiny_pools(_small(scenes.disc2d(1), 256))),
    ("arm6-capacity", lambda: _tiny_pools(_small(scenes.arm6(2), 512, groups=8))),
    # the root-recycling workload at its own shape: 7 DOF, 60 spheres, 32
    # obstacles on 16 waypoints, 64 slots, 8192 samples per iteration
    ("arm7-rr-full", lambda: scenes.arm7rr(2)),
    # the 6-DOF arm workload at its own shape (4096 samples per iteration,
    # the launch shapes the benchmark times)
    ("arm6-ir-full", lambda: scenes.arm6(2)),
]
# largest fraction of workers with an exempt decision that may end differently
# (measured on MI355X: at most 0.83 %, disc2d-rr; 0 of 4452 exempt workers in
# the grazing case)
MAX_EXEMPT_DIFF = 0.02


@pytest.mark.parametrize("name,make", PROBS, ids=[p[0] for p in PROBS])
def test_sampling_matches_oracle(oracle_lib, name, make):
    from paper_2609_30533_amd.lib import Problem
    prob = make()
    banner("sample %s" % name)
    gp = Problem(prob)
    op = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    B = prob.params.batch
    for it in (0, 1, 7):
        s = _to_np(gp.sample(it))
        r = op.sample(it, B)
        assert np.array_equal(s["dir"], r["dir"])
        assert np.array_equal(s["grp"], r["grp"])
        np.testing.assert_allclose(s["qr"], r["qr"], rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(s["T"], r["T"], rtol=1e-6, atol=1e-6)
        diff = np.where(s["flags"] != r["flags"])[0]
        for i in diff:
            # only fragile root checks or a near-empty Eq. 6 interval may differ
            _, m = o.state_valid(np.r_[prob.q_goal, r["T"][i]])
            q = r["qr"][:, i]
            lo = np.linalg.norm(q - prob.q_start) / prob.v_max
            hi = r["T"][i] - np.linalg.norm(q - prob.q_goal) / prob.v_max
            assert abs(m) <= MARGIN or abs(hi - lo) <= 1e-5 * max(1.0, abs(hi)), (i, s["flags"][i], r["flags"][i])
        assert len(diff) <= 0.01 * B
        ok = (s["flags"] & 1) == 0
        np.testing.assert_allclose(s["tr"][ok], r["tr"][ok], rtol=1e-5, atol=2e-5)


def _compare_batch(prob, s, g, r, counts=None):
    """Compare one extend batch.  Returns (exempt workers, exempt workers whose
    outcome differs); non-exempt workers must agree.  counts: pool sizes
    before the batch.  Once an exempt worker of a pool has ended differently,
    the nodes appended to that pool in this batch (fresh virtual roots among
    them) have different indices on the two sides, so a parent appended in
    this batch is only required to be new on both sides."""
    B = len(s["dir"])
    P = prob.params

    def appended(pool, idx):
        base = 0 if pool == 0 else P.cap_fwd + (pool - 1) * P.cap_bwd
        return counts is not None and idx - base >= counts[pool]
    exempt = (r["amb"] != 0) | (r["edge_margin"] <= MARGIN) | (r["bridge_margin"] <= MARGIN)
    skip = (s["flags"] & 1) != 0
    n_ex = n_ex_diff = 0
    pool_diverged = set()
    for w in range(B):
        if skip[w]:
            assert g["status"][w] == 0 and r["status"][w] == 0
            continue
        pool = 0 if s["dir"][w] == 0 else 1 + s["grp"][w]
        if exempt[w]:
            n_ex += 1
            ok_r = r["bridge_ok"][w] if (r["status"][w] == 2 and r["bridge"][w] >= 0) else 0
            # a trapped worker has no parent in Alg. 1's result (the oracle
            # reports -1, the device the nearest node it started from)
            diff = (g["status"][w] != r["status"][w] or
                    (r["status"][w] >= 2 and g["parent"][w] != r["parent"][w]) or
                    (r["status"][w] == 2 and (g["bridge"][w] != r["bridge"][w] or g["bridge_ok"][w] != ok_r)))
            if diff:
                n_ex_diff += 1
                pool_diverged.add(pool)
            continue
        if pool in pool_diverged and g["status"][w] in (2, 3) and r["status"][w] in (2, 3):
            # an earlier exempt worker of this pool claimed a different number
            # of slots on the two sides, so where the pool fills up the
            # claims of later workers end at different offsets
            if g["status"][w] != r["status"][w]:
                continue
        else:
            assert g["status"][w] == r["status"][w], (w, g["status"][w], r["status"][w])
        if r["status"][w] < 2:
            continue
        if pool in pool_diverged and appended(pool, r["parent"][w]):
            assert appended(pool, g["parent"][w]), (w, g["parent"][w], r["parent"][w])
        else:
            assert g["parent"][w] == r["parent"][w], (w, g["parent"][w], r["parent"][w])
        np.testing.assert_allclose(g["xnew"][:, w], r["xnew"][:, w], rtol=1e-5, atol=2e-5)
        if pool not in pool_diverged:
            assert g["new_idx"][w] == r["new_idx"][w], (w, g["new_idx"][w], r["new_idx"][w])
        if r["status"][w] != 2:
            continue
        assert g["bridge"][w] == r["bridge"][w], (w, g["bridge"][w], r["bridge"][w])
        ok_r = r["bridge_ok"][w] if r["bridge"][w] >= 0 else 0
        assert g["bridge_ok"][w] == ok_r, (w, g["bridge_ok"][w], ok_r)
        if ok_r:
            assert abs(g["Up"][w] - r["Up"][w]) <= 1e-5 * max(1.0, r["Up"][w])
            assert abs(g["Cp"][w] - r["Cp"][w]) <= 1e-5 * max(1.0, r["Cp"][w]) + 2e-5
    return n_ex, n_ex_diff


@pytest.mark.parametrize("name,make", PROBS, ids=[p[0] for p in PROBS])
def test_extend_lockstep_resync(oracle_lib, name, make):
    from paper_2609_30533_amd.lib import Problem
    prob = make()
    banner("extend %s" % name)
    gp = Problem(prob)
    op = oracle_lib.Planner(prob)
    total_ex = total_diff = total = n_dropped = 0
    for it in range(12):
        st = _resync(gp, op, prob)
        s_dev = gp.sample(it)
        s = _to_np(s_dev)
        g = _to_np(gp.extend(s_dev))
        sr = dict(dir=s["dir"], flags=s["flags"], grp=s["grp"], T=s["T"].astype(np.float64),
                  qr=s["qr"].astype(np.float64), tr=s["tr"].astype(np.float64))
        r = op.extend(sr)
        n_ex, n_diff = _compare_batch(prob, s, g, r, st["counts"])
        total_ex += n_ex
        total_diff += n_diff
        total += int(((s["flags"] & 1) == 0).sum())
        gi, oi = gp.info(), op.info()
        if n_diff == 0:
            # same decisions: same incumbent and the same pool sizes
            if math.isfinite(oi["U"]):
                assert abs(gi["U"] - oi["U"]) <= 1e-5 * max(1.0, oi["U"])
                assert abs(gi["C"] - oi["C"]) <= 1e-5 * max(1.0, oi["C"]) + 2e-5
            else:
                assert not math.isfinite(gi["U"])
            assert np.array_equal(gp.export()["counts"], op.counts())
            assert bool(gi["overflow"]) == bool(oi["overflow"])
        n_dropped += int((g["status"] == 3).sum())
    if name.endswith("capacity"):
        assert n_dropped > 0, "the pools never filled up"
    banner("%s: %d workers, %d exempt, %d exempt with a different outcome, %d dropped" % (
        name, total, total_ex, total_diff, n_dropped))
    assert total > 0
    assert total_ex <= 0.5 * total
    assert total_diff <= MAX_EXEMPT_DIFF * total, (total_diff, total)


PLAN_CASES = [
    # (name, problem, iterations, must solve)
    ("disc2d-ir-0", lambda: _small(scenes.disc2d(0), 512), 60, True),
    ("disc2d-ir-2", lambda: _small(scenes.disc2d(2), 512), 60, True),
    ("disc2d-ir-3", lambda: _small(scenes.disc2d(3), 512), 60, True),
    ("disc2d-rr-0", lambda: _small(scenes.disc2d(0, params=scenes.Params(variant=1, n_groups=8)), 512), 60, True),
    ("disc2d-rr-2", lambda: _small(scenes.disc2d(2, params=scenes.Params(variant=1, n_groups=8)), 512), 60, True),
    ("arm6-ir-2", lambda: _small(scenes.arm6(2), 1024, groups=8), 200, True),
    # start and goal redrawn until the library accepts them (the attempt index
    # found by that redraw), pools large enough for the iterations
    ("arm7-rr-5", lambda: _small(scenes.arm7rr(5, n_obs=8, attempt=1), 1024, 1 << 16, 1 << 13, 16), 400, True),
    ("arm7-rr-8", lambda: _small(scenes.arm7rr(8, n_obs=8, attempt=3), 1024, 1 << 16, 1 << 13, 16), 400, True),
    ("arm6-static-ir-14", lambda: _small(scenes.arm6static(14, attempt=42), 1024, 1 << 16, 1 << 13, 8), 600, True),
    ("arm6-static-ir-24", lambda: _small(scenes.arm6static(24, attempt=9), 1024, 1 << 16, 1 << 13, 8), 600, True),
    # the recycling workload's full shape (start and goal accepted at attempt 0)
    ("arm7-rr-c3-22", lambda: _c3_parked(22), 40, True),
    ("arm7-rr-c3-26", lambda: _c3_parked(26), 40, True),
]


@pytest.mark.parametrize("name,make,iters,must", PLAN_CASES, ids=[c[0] for c in PLAN_CASES])
def test_plan_paths_validate(oracle_lib, name, make, iters, must):
    from paper_2609_30533_amd.lib import Problem
    prob = make()
    banner("plan %s" % name)
    o = oracle_lib.Oracle(prob)
    gp = Problem(prob)
    res = gp.plan(max_iters=iters, iters_per_sync=4)
    inf = gp.info()
    banner("%s: rc %d U %.4f C %.4f first iter %d first %.2f ms total %.2f ms iters %d" % (
        name, res["rc"], res["U"], res["C"], res["first_iter"], res["first_ms"], res["total_ms"], res["iterations"]))
    if must:
        assert res["rc"] == 0
    if res["rc"] == 0:
        ok, msg = o.validate_path(res["states"], res["U"], res["C"], rel_tol=1e-4)
        assert ok, msg
        assert res["U"] >= inf["L"] - 1e-5
        assert res["first_iter"] >= 0 and res["first_ms"] > 0
        # device time of the iterations up to the first solution, inside the
        # call's wall time (which adds the start check and the graph capture)
        assert res["first_ms"] <= res["total_ms"]


def test_roots_update_after_improvement(oracle_lib):
    """After a strict drop of U every active recycling root lies below U and
    every recycled slot holds a valid root in [L_grid, U)."""
    from paper_2609_30533_amd.lib import Problem
    prob = _small(scenes.disc2d(2, params=scenes.Params(variant=1, n_groups=8)), 512)
    gp = Problem(prob)
    o = oracle_lib.Oracle(prob)
    prev_gen = gp.slots()[2].copy()
    for it in range(30):
        gp.iterate(1)
        inf = gp.info()
        T, act, gen, k = gp.slots()
        assert np.all(gen >= prev_gen)
        if math.isfinite(inf["U"]):
            assert np.all(T[act == 1] < inf["U"])
            for sl in np.where(gen > prev_gen)[0]:
                assert T[sl] < inf["U"] and o.state_valid(np.r_[prob.q_goal, T[sl]])[0]
        prev_gen = gen.copy()


def test_interval_root_partition_matches_oracle(oracle_lib):
    from paper_2609_30533_amd.lib import Problem
    prob = _small(scenes.arm6(3), 256)
    gp = Problem(prob)
    op = oracle_lib.Planner(prob)
    I1, p1 = gp.partition()
    I2, p2 = op.partition()
    np.testing.assert_allclose(I1, I2, rtol=1e-12, atol=1e-12)
    for a, b in zip(p1, p2):
        assert a.shape == b.shape
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_invalid_arguments_are_errors():
    from paper_2609_30533_amd import lib
    prob = scenes.disc2d(0)
    prob.t_min = 11.0   # t_min > t_max
    with pytest.raises(lib.StError):
        lib.Problem(prob)
    prob = scenes.disc2d(0)
    prob.v_max = 0.0
    with pytest.raises(lib.StError):
        lib.Problem(prob)
    prob = scenes.disc2d(0)
    prob.q_start = np.array([2.0, 0.5])    # outside C
    with pytest.raises(lib.StError):
        lib.Problem(prob)
    torch_cuda()


@pytest.mark.parametrize("make", [lambda: _small(scenes.arm6(2), 1024, groups=8),
                                  lambda: _small(scenes.disc2d(0), 512)], ids=["arm6", "disc2d"])
def test_extension_paths_agree(make):
    """The flattened and the chunked extension-edge paths decide identically,
    so the planner's trees after some iterations are equal bit for bit."""
    from paper_2609_30533_amd.lib import Problem
    torch = torch_cuda()
    prob = make()
    banner("extension paths %s" % prob.name)
    states = []
    for epb in (0, 1, 2, 8):
        gp = Problem(prob)
        gp.set_flat_extension(epb)
        gp.iterate(12)
        torch.cuda.synchronize()
        st = gp.export()
        c = st["counts"]
        p = prob.params
        rows = np.concatenate([np.arange(0 if k == 0 else p.cap_fwd + (k - 1) * p.cap_bwd,
                                         (0 if k == 0 else p.cap_fwd + (k - 1) * p.cap_bwd) + int(n))
                               for k, n in enumerate(c)])
        states.append((c, st["x"][rows], st["parent"][rows], gp.work_counters()))
        gp.close()
    for c, x, par, w in states[1:]:
        assert np.array_equal(c, states[0][0])
        assert np.array_equal(x, states[0][1])
        assert np.array_equal(par, states[0][2])
        assert w["edges"] == states[0][3]["edges"] and w["edge_states"] == states[0][3]["edge_states"]


def _iterate_until_solved(gp, max_iters):
    for it in range(max_iters):
        gp.iterate(1)
        inf = gp.info()
        if math.isfinite(inf["U"]):
            return it + 1, inf
    return max_iters, gp.info()


@pytest.mark.parametrize("name,make", [
    ("disc2d-ir", lambda: _small(scenes.disc2d(3, t_min=0.0), 512)),
    ("arm6-ir", lambda: _small(scenes.arm6(2), 1024, groups=8)),
], ids=["disc2d-ir", "arm6-ir"])
def test_interval_root_after_improvement(oracle_lib, name, make):
    """Alg. 2's update on a drop of U, done by the device inside the publish
    step: the repartition below Ubar = min(H, U) (uniform intervals and
    guided shares, Sec. IV-B, Fig. 2(b)) equals the oracle's; the next
    samples (root times drawn from the new partition, groups without an
    active tree) equal the oracle's; the next extend batch, where trees
    rooted at T >= U no longer take part, agrees in lockstep."""
    from paper_2609_30533_amd.lib import Problem
    prob = make()
    banner("interval root after improvement %s" % name)
    gp = Problem(prob)
    op = oracle_lib.Planner(prob)
    o = oracle_lib.Oracle(prob)
    n, inf = _iterate_until_solved(gp, 300)
    assert math.isfinite(inf["U"]), "no incumbent within 300 iterations"
    banner("%s: U %.6f after %d iterations (L %.4f, H %.4f)" % (name, inf["U"], n, inf["L"], inf["H"]))
    assert inf["U"] < inf["H"]
    st = _resync(gp, op, prob)
    I1, p1 = gp.partition()
    I2, p2 = op.partition()
    np.testing.assert_allclose(I1, I2, rtol=1e-12, atol=1e-12)
    assert abs(I1[-1, 1] - min(inf["H"], inf["U"])) < 1e-12
    for a, b in zip(p1, p2):
        assert a.shape == b.shape
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
    # the groups' guided shares are equal and lie below Ubar
    q = [float((pc[:, 1] - pc[:, 0]).sum()) if len(pc) else 0.0 for pc in p1]
    assert np.allclose(q, q[0], atol=1e-9)
    assert all(pc[:, 1].max() <= inf["U"] + 1e-12 for pc in p1 if len(pc))
    B = prob.params.batch
    it = int(inf["iter"])
    s = _to_np(gp.sample(it))
    r = op.sample(it, B)
    assert np.array_equal(s["dir"], r["dir"]) and np.array_equal(s["grp"], r["grp"])
    np.testing.assert_allclose(s["T"], r["T"], rtol=1e-6, atol=1e-6)
    assert np.all(s["T"] < inf["U"] + 1e-6)
    diff = np.where(s["flags"] != r["flags"])[0]
    for i in diff:
        _, m = o.state_valid(np.r_[prob.q_goal, r["T"][i]])
        qq = r["qr"][:, i]
        lo = np.linalg.norm(qq - prob.q_start) / prob.v_max
        hi = r["T"][i] - np.linalg.norm(qq - prob.q_goal) / prob.v_max
        assert abs(m) <= MARGIN or abs(hi - lo) <= 1e-5 * max(1.0, abs(hi)), (i, s["flags"][i], r["flags"][i])
    assert len(diff) <= 0.01 * B
    # one extend batch after the drop, in lockstep
    s_dev = gp.sample(it)
    s = _to_np(s_dev)
    g = _to_np(gp.extend(s_dev))
    sr = dict(dir=s["dir"], flags=s["flags"], grp=s["grp"], T=s["T"].astype(np.float64),
              qr=s["qr"].astype(np.float64), tr=s["tr"].astype(np.float64))
    rr = op.extend(sr)
    n_ex, n_diff = _compare_batch(prob, s, g, rr, st["counts"])
    banner("%s: after-drop batch, %d exempt, %d differing" % (name, n_ex, n_diff))
    assert n_diff <= 0.05 * B


def test_interval_root_termination(oracle_lib):
    """Alg. 2 stops once L >= min(H, U): with an incumbent at U = L imported
    into both sides, no worker runs (every sample is skipped, the trees do
    not change) and the planning loop returns at its first check."""
    from paper_2609_30533_amd.lib import Problem
    prob = _small(scenes.disc2d(3, t_min=0.0), 512)
    gp = Problem(prob)
    op = oracle_lib.Planner(prob)
    n, inf = _iterate_until_solved(gp, 300)
    assert math.isfinite(inf["U"])
    st = gp.export()
    L = inf["L"]
    gp.import_state(st["counts"], st["x"], st["parent"], st["cost"], st["rootT"], L, inf["C"], inf["inc_fwd"],
                    inf["inc_bwd"], inf["iter"])
    op.import_state(st["counts"], st["x"].astype(np.float64), st["parent"], st["cost"].astype(np.float64),
                    st["rootT"].astype(np.float64), L, inf["C"], inf["inc_fwd"], inf["inc_bwd"], inf["iter"])
    s = _to_np(gp.sample(int(inf["iter"])))
    r = op.sample(int(inf["iter"]))
    assert np.all(s["flags"] & 1) and np.all(r["flags"] & 1)
    gp.iterate(8)
    assert np.array_equal(gp.export()["counts"], st["counts"])
    it0 = op.info()["iter"]
    op.run(8)
    assert op.info()["iter"] == it0
    it_before = gp.info()["iter"]
    res = gp.plan(max_iters=400, iters_per_sync=4)
    assert res["iterations"] <= it_before + 4
    assert np.array_equal(gp.export()["counts"], st["counts"])


def test_trivial_case_on_device(oracle_lib):
    """q_s = q_g with a free start and arrival at time 0 allowed is the
    trivial case (Alg. 2 / Alg. 3 return the one-state path); with the
    arrival range starting later the problem is planned as usual."""
    from paper_2609_30533_amd import lib
    for variant in (0, 1):
        prob = scenes.disc2d(0, params=scenes.Params(variant=variant, n_groups=4 if variant == 0 else 8))
        _small(prob, 256)
        prob.q_goal = prob.q_start.copy()
        prob.t_min = 0.0
        prob.wp[:, :, 1:3] = 50.0
        gp = lib.Problem(prob)
        res = gp.plan(max_iters=20, iters_per_sync=4)
        assert res["rc"] == lib.ST_TRIVIAL
        assert res["states"].shape == (1, 3) and res["U"] == 0.0 and res["C"] == 0.0
        assert oracle_lib.Planner(prob).run(5) == 2
        prob.t_min = 2.0
        gp2 = lib.Problem(prob)
        res2 = gp2.plan(max_iters=80, iters_per_sync=4)
        assert res2["rc"] == 0 and res2["U"] >= 2.0
        ok, msg = oracle_lib.Oracle(prob).validate_path(res2["states"], res2["U"], res2["C"], rel_tol=1e-4)
        assert ok, msg


def test_capacity_exhausted_is_reported(oracle_lib):
    """Pools too small for any path: the planner drops inserts, reports the
    overflow, and st_plan ends with ST_ECAPACITY instead of a silent
    failure; the trees stay within their capacities."""
    from paper_2609_30533_amd import lib
    prob = _small(scenes.arm6(2), 512, cap_f=24, cap_b=6, groups=8)
    gp = lib.Problem(prob)
    res = gp.plan(max_iters=24, iters_per_sync=4)
    inf = gp.info()
    assert inf["overflow"] == 1
    assert res["rc"] == lib.ST_ECAPACITY and res["states"] is None
    c = gp.export()["counts"]
    assert c[0] <= 24 and np.all(c[1:] <= 6)


@pytest.mark.parametrize("name,make", [
    ("arm6-ir", lambda: _small(scenes.arm6(2), 1024, 1 << 15, 1 << 12, 8)),
    ("arm7-rr", lambda: _small(scenes.arm7rr(2, n_obs=16), 1024, 1 << 15, 1 << 12, 16)),
    ("disc2d-ir", lambda: _small(scenes.disc2d(3), 512)),
    ("arm6-ir-full", lambda: scenes.arm6(2)),
], ids=["arm6-ir", "arm7-rr", "disc2d-ir", "arm6-ir-full"])
def test_iterate_equals_sample_and_extend(name, make):
    """The planner's own iterations (the sampler buckets its workers by node
    set, the extend step runs without the separate bucketing kernel, graph
    replays) and the same iterations through st_sample_batch +
    st_extend_batch (caller-given samples, bucketed by k_prep) build the same
    trees, node for node, and the same incumbent."""
    from paper_2609_30533_amd.lib import Problem
    torch = torch_cuda()
    banner("iterate vs sample+extend %s" % name)
    ga, gb = Problem(make()), Problem(make())
    n = 12
    ga.iterate(n)
    for it in range(n):
        gb.extend(gb.sample(it))
    torch.cuda.synchronize()
    ea, eb = ga.export(), gb.export()
    assert np.array_equal(ea["counts"], eb["counts"]), (ea["counts"], eb["counts"])
    assert ea["counts"].sum() > 0
    prm = ga.prob.params
    for p, c in enumerate(ea["counts"]):
        base = 0 if p == 0 else prm.cap_fwd + (p - 1) * prm.cap_bwd
        for k in ("x", "parent", "cost", "rootT"):
            assert np.array_equal(ea[k][base:base + c], eb[k][base:base + c]), (k, p)
    ia, ib = ga.info(), gb.info()
    assert ia["U"] == ib["U"] and ia["C"] == ib["C"] and ia["iter"] == ib["iter"] == n


def test_recycling_initial_roots_worked_example():
    """The library's initial recycling roots on the hand-worked scene of
    tests/golden/rr_worked_example.txt (reading 12) equal the values derived
    by hand, as the oracle's do."""
    from paper_2609_30533_amd.lib import Problem
    from tests import oracle_pins
    torch_cuda()
    prob, rows = oracle_pins.rr_worked_problem()
    gp = Problem(prob)
    T, act, gen, k = gp.slots()
    assert np.array_equal(k, [int(v) for v in rows["init.k"].split()]), k
    assert np.allclose(T, [float(v) for v in rows["init.T"].split()], atol=1e-6), T
    assert np.array_equal(act, [int(v) for v in rows["init.active"].split()]), act
    assert np.array_equal(gen, [0, 0, 0, 0]), gen
