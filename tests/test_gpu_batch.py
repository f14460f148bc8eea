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
    from paper_2609_30533_amd.lib import Batch, Problem
    torch = torch_cuda()
    probs = _members()
    banner("batch parity: %d members" % len(probs))
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
