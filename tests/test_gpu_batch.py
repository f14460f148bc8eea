"""The many-problem launch sequence against the same problems run one by one.

The kernels of a batch are the single-problem kernels reading their launch
record from device memory, and every decision of the pipeline is independent
of the launch shape (nearest nodes and bridges are exact minima over
(key, index), first hits are minima over state indices, inserts follow the
worker order), so after the same number of iterations every member's trees
and incumbent must equal those of the problem run alone, bit for bit.  Paths
found by a batch are re-validated by the oracle."""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu


def _shrink(prob, batch, cap_f, cap_b, groups=None):
    prob.params.batch = batch
    prob.params.cap_fwd = cap_f
    prob.params.cap_bwd = cap_b
    if groups:
        prob.params.n_groups = groups
    return prob


def _members():
    probs = [
        _shrink(scenes.disc2d(0), 256, 1 << 14, 1 << 12),
        _shrink(scenes.disc2d(3), 96, 1 << 13, 1 << 11),
        _shrink(scenes.arm6(2), 512, 1 << 15, 1 << 12),
        _shrink(scenes.disc2d(2, params=scenes.Params(variant=1, n_groups=8)), 128, 1 << 14, 1 << 11),
        _shrink(scenes.arm7rr(2, n_obs=8), 320, 1 << 15, 1 << 11, groups=16),
        _shrink(scenes.arm6static(7), 256, 1 << 15, 1 << 12),
        # 65 pools for 64 samples: the insertion blocks of the single runs
        # have fewer threads than pools
        _shrink(scenes.arm7rr(11, n_obs=8), 64, 1 << 14, 1 << 10, groups=64),
    ]
    for s in range(3):
        m = scenes.mixed(100 + s)
        probs.append(_shrink(m, 64 + 32 * s, min(m.params.cap_fwd, 1 << 15), min(m.params.cap_bwd, 1 << 12)))
    return probs


def _state(gp):
    """Used node slots of every pool (unused slots hold whatever the device
    memory held) and the planner info."""
    st = gp.export()
    inf = gp.info()
    p = gp.prob.params
    used = []
    for k, c in enumerate(st["counts"]):
        base = 0 if k == 0 else p.cap_fwd + (k - 1) * p.cap_bwd
        used.append(np.arange(base, base + int(c)))
    idx = np.concatenate(used) if used else np.zeros(0, dtype=np.int64)
    return {"counts": st["counts"], "x": st["x"][idx], "parent": st["parent"][idx], "cost": st["cost"][idx],
            "rootT": st["rootT"][idx]}, inf


def test_batch_equals_single_runs(oracle_lib):
    _batch_vs_single(oracle_lib, _members(), "batch parity")


def test_small_sample_batch_equals_single_runs(oracle_lib):
    # at most 64 samples per member: the batch scans in tiles of 64 queries
    # (one-wave blocks) while the single runs keep tiles of 256
    probs = _members()
    for i, p in enumerate(probs):
        p.params.batch = (32, 48, 64)[i % 3]
    _batch_vs_single(oracle_lib, probs, "small-sample batch parity")


def _batch_vs_single(oracle_lib, probs, what):
    from paper_2609_30533_amd.lib import Batch, Problem
    torch = torch_cuda()
    banner("%s: %d members" % (what, len(probs)))
    single = [Problem(p, problem_id=i) for i, p in enumerate(probs)]
    mem = [Problem(p, problem_id=i) for i, p in enumerate(probs)]
    batch = Batch(mem, iters_per_launch=4)
    iters = 12
    batch.iterate(iters)
    for gp in single:
        gp.iterate(iters)
    torch.cuda.synchronize()
    launched = 0
    for i, (a, b) in enumerate(zip(single, mem)):
        sa, ia = _state(a)
        sb, ib = _state(b)
        start_ok, m = oracle_lib.Oracle(probs[i]).state_valid(np.r_[probs[i].q_start, 0.0])
        if not start_ok and abs(m) > 1e-4:
            assert ib["iter"] == 0, i  # a colliding start takes no part in the launches
            continue
        if ib["iter"] == 0 and abs(m) <= 1e-4:
            continue  # grazing start: the device may decide either way
        launched += 1
        assert ia["iter"] == ib["iter"], (i, ia["iter"], ib["iter"])
        assert np.array_equal(sa["counts"], sb["counts"]), (i, sa["counts"], sb["counts"])
        assert np.array_equal(sa["x"], sb["x"]), i
        assert np.array_equal(sa["parent"], sb["parent"]), i
        assert np.array_equal(sa["cost"], sb["cost"]), i
        assert np.array_equal(sa["rootT"], sb["rootT"]), i
        assert (ia["U"] == ib["U"]) or (math.isinf(ia["U"]) and math.isinf(ib["U"])), i
        assert ia["first_iter"] == ib["first_iter"], i
    assert launched >= 5, launched
    batch.close()


def test_batch_plan_paths_validate(oracle_lib):
    from paper_2609_30533_amd.lib import Batch, Problem
    torch_cuda()
    probs = [_shrink(scenes.disc2d(s), 128, 1 << 15, 1 << 13) for s in range(8)]
    banner("batch plan: %d disc problems" % len(probs))
    mem = [Problem(p, problem_id=i) for i, p in enumerate(probs)]
    batch = Batch(mem)
    r = batch.plan(max_ms=3000, stop_at_first=True)
    assert r["iterations"] > 0
    solved = 0
    for i, (p, gp) in enumerate(zip(probs, mem)):
        o = oracle_lib.Oracle(p)
        start_ok, _ = o.state_valid(np.r_[p.q_start, 0.0])
        if not start_ok:
            assert r["first_iter"][i] == -1 and math.isnan(r["first_ms"][i])
            continue
        if r["first_iter"][i] < 0:
            assert math.isnan(r["first_ms"][i]) and math.isinf(r["U"][i])
            continue
        solved += 1
        assert r["first_ms"][i] > 0
        path = gp.path()
        assert path["rc"] == 0 and path["states"] is not None
        assert abs(path["U"] - r["U"][i]) <= 1e-6 * max(1.0, r["U"][i])
        ok, msg = o.validate_path(path["states"], path["U"], path["C"], rel_tol=1e-4)
        assert ok, (i, msg)
    assert solved >= 5, solved
    assert r["n_solved"] == solved
    batch.close()


def test_batch_rejects_changed_members():
    from paper_2609_30533_amd.lib import Batch, Problem, StError
    torch_cuda()
    p = _shrink(scenes.disc2d(0), 64, 1 << 12, 1 << 10)
    gp = Problem(p)
    batch = Batch([gp])
    batch.iterate(4)
    # growing the member's own sample count reallocates its work buffers
    gp.sample(0, B=4096)
    s = gp.sample(0, B=4096)
    gp.extend(s)
    with pytest.raises(StError):
        batch.iterate(4)
    batch.close()
    with pytest.raises(StError):
        Batch([gp, gp])


def _pool_slice(prob, pool, lo, hi):
    P = prob.params
    base = 0 if pool == 0 else P.cap_fwd + (pool - 1) * P.cap_bwd
    return np.arange(base + lo, base + hi)


def test_c4_batch_lockstep_and_paths(oracle_lib):
    """512 heterogeneous problems (DOF 2/6/7, 4-64 obstacles, arrival widths
    5-60 s, capacities 2^14-2^18) in one batch: for members of every DOF and
    capacity class, each batched iteration equals the oracle's extend step on
    the member's state before it (resynchronised lockstep: the same pool
    counts, the same new nodes and parents, the same incumbent, unless the
    oracle flags a numerically fragile decision of that iteration); then the
    batch plans within a budget and every path it finds is re-validated by
    the oracle."""
    from paper_2609_30533_amd.lib import Batch, Problem
    torch = torch_cuda()
    n = 512
    probs = [scenes.mixed(s) for s in range(n)]
    banner("c4 batch: %d members" % n)
    mem = [Problem(p, problem_id=i) for i, p in enumerate(probs)]
    batch = Batch(mem, iters_per_launch=1)
    batch.iterate(1)
    torch.cuda.synchronize()
    launched = [i for i in range(n) if mem[i].info()["iter"] == 1]
    assert len(launched) >= 100, len(launched)  # members whose start collides take no part
    # members to follow: for each DOF, the smallest and the largest forward capacity
    pick = []
    for d in (2, 6, 7):
        cand = sorted([i for i in launched if probs[i].d == d], key=lambda i: probs[i].params.cap_fwd)
        assert cand, d
        pick += [cand[0], cand[-1]] if len(cand) > 1 else cand[:1]
    banner("c4 batch: following members %s (caps %s)" % (pick, [probs[i].params.cap_fwd for i in pick]))
    planners = {i: oracle_lib.Planner(probs[i], problem_id=i) for i in pick}
    agree = fragile = 0
    for it in range(1, 7):
        pre = {}
        for i in pick:
            slots = mem[i].slots() if probs[i].params.variant == 1 else None
            pre[i] = (mem[i].export(), mem[i].info(), slots)
        batch.iterate(1)
        torch.cuda.synchronize()
        for i in pick:
            st, inf, slots = pre[i]
            op = planners[i]
            op.import_state(st["counts"], st["x"].astype(np.float64), st["parent"], st["cost"].astype(np.float64),
                            st["rootT"].astype(np.float64), inf["U"], inf["C"], inf["inc_fwd"], inf["inc_bwd"],
                            inf["iter"], slots)
            s = op.sample(int(inf["iter"]))
            r = op.extend(s)
            post = mem[i].export()
            pinf = mem[i].info()
            same_counts = np.array_equal(post["counts"], op.counts())
            risky = bool((r["amb"] != 0).any() or (r["edge_margin"] <= 1e-4).any() or
                         (r["bridge_margin"] <= 1e-4).any() or ((s["flags"] & 1) == 0).sum() == 0)
            if not same_counts:
                assert risky, (i, it, post["counts"], op.counts())
                fragile += 1
                continue
            oe = op.export()
            for pool, (c0, c1) in enumerate(zip(st["counts"], post["counts"])):
                if c1 == c0:
                    continue
                idx = _pool_slice(probs[i], pool, int(c0), int(c1))
                if not np.array_equal(post["parent"][idx], oe["parent"][idx]):
                    assert risky, (i, it, pool)
                    fragile += 1
                    break
                np.testing.assert_allclose(post["x"][idx], oe["x"][idx], rtol=1e-5, atol=2e-5)
                np.testing.assert_allclose(post["cost"][idx], oe["cost"][idx], rtol=1e-5, atol=2e-5)
            else:
                oi = op.info()
                if math.isfinite(oi["U"]):
                    assert abs(pinf["U"] - oi["U"]) <= 1e-5 * max(1.0, oi["U"]), (i, it)
                else:
                    assert not math.isfinite(pinf["U"]), (i, it)
                agree += 1
    banner("c4 batch lockstep: %d member-iterations agree, %d with a fragile decision" % (agree, fragile))
    assert agree >= 0.8 * (agree + fragile) and agree > 0
    # plan within a budget; every solved member's path is re-validated
    r = batch.plan(max_ms=1500)
    solved = 0
    for i in range(n):
        if r["first_iter"][i] < 0:
            continue
        path = mem[i].path()
        assert path["rc"] == 0 and path["states"] is not None, i
        ok, msg = oracle_lib.Oracle(probs[i], problem_id=i).validate_path(path["states"], path["U"], path["C"],
                                                                          rel_tol=1e-4)
        assert ok, (i, msg)
        solved += 1
    banner("c4 batch plan: %d of %d members solved in %d iterations, every path valid" % (
        solved, n, r["iterations"]))
    assert solved == r["n_solved"] and solved >= 20
    batch.close()


def test_autotuner_table_is_honoured(tmp_path):
    """autotune.py tunes one class on the device, writes its table as JSON,
    and the table read back sets each problem's samples per iteration and
    launch shape, which a batch of those problems then runs with."""
    from paper_2609_30533_amd import autotune
    from paper_2609_30533_amd.lib import Batch, Problem
    torch = torch_cuda()
    out = tmp_path / "tuning.json"
    rc = autotune.main(["--out", str(out), "--problems", "6", "--budget-ms", "25", "--keys", "d2-o8,d6-o16"])
    assert rc == 0 and out.exists()
    table = autotune.load(str(out))
    assert set(table) == {"d2-o8", "d6-o16"}
    for e in table.values():
        assert e["samples"] in autotune.SAMPLES and e["lanes_bridge"] in autotune.LANES
    for key in table:
        probs = autotune.tuning_problems(key, 3, seed0=7_000_000)
        gps = []
        for p in probs:
            autotune.apply(p, table)
            g = Problem(p)
            autotune.apply(p, table, g)
            inf = g.info()
            assert inf["batch"] == table[key]["samples"]
            assert inf["lanes_bridge"] == table[key]["lanes_bridge"]
            assert inf["lanes_extension"] == table[key]["lanes_extension"]
            gps.append(g)
        b = Batch(gps)
        w0 = [g.work_counters()["edges"] for g in gps]
        b.iterate(4)
        torch.cuda.synchronize()
        for g, e0 in zip(gps, w0):
            inf = g.info()
            if inf["iter"] == 0:
                continue  # colliding start: not launched
            assert inf["iter"] == 4
            # at most one extension edge per worker and iteration
            assert g.work_counters()["edges"] - e0 <= 4 * table[key]["samples"]
        b.close()


def test_batch_rejects_too_many_samples():
    from paper_2609_30533_amd.lib import Batch, Problem, StError
    torch_cuda()
    # a member's samples index a grid dimension of the batched bridge check
    p = _shrink(scenes.disc2d(0), 65536, 1 << 12, 1 << 10)
    gp = Problem(p)
    with pytest.raises(StError, match="samples per iteration"):
        Batch([gp])
    gp.close()
