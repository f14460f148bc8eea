"""Goal sequences (Sec. III): successive single-goal queries with local time
reset and obstacle trajectories shifted by the previous arrival.  Every
returned path is re-validated by the oracle in absolute time against the
original, unshifted scene."""
import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu


def _goals(prob, m, seed):
    rng = np.random.default_rng([11, seed])
    r = float(prob.sphere[0, 3])
    g = [scenes.f32(rng.uniform(r, 1.0 - r, size=2)) for _ in range(m - 1)]
    return np.array(g + [prob.q_goal])


def _validate(oracle_lib, prob, states, goals, U):
    o = oracle_lib.Oracle(prob)
    d = prob.d
    assert np.allclose(states[0, :d], prob.q_start, atol=1e-6) and abs(states[0, d]) < 1e-9
    assert np.all(np.diff(states[:, d]) > 0)
    D = np.linalg.norm(np.diff(states[:, :d], axis=0), axis=1)
    assert np.all(D <= prob.v_max * np.diff(states[:, d]) * (1 + 1e-5) + 1e-9)
    res = o.check_edges(states[:-1], states[1:])
    assert np.all(res["free"] == 1), np.where(res["free"] == 0)
    # the goals are visited in order
    k = 0
    for g in goals:
        while k < len(states) and not np.allclose(states[k, :d], g, atol=1e-6):
            k += 1
        assert k < len(states), "goal not visited in order"
    assert np.allclose(states[-1, :d], goals[-1], atol=1e-6)
    assert abs(states[-1, d] - U) <= 1e-6 * max(1.0, U) and U <= prob.t_max + 1e-6


def test_goal_sequences_validate(oracle_lib):
    from paper_2609_30533_amd.lib import plan_sequence
    torch_cuda()
    ok = 0
    for seed in (0, 2, 3):
        prob = scenes.disc2d(seed)
        prob.params.batch = 512
        goals = _goals(prob, 3, seed)
        banner("sequence disc2d seed %d" % seed)
        r = plan_sequence(prob, goals, max_iters=300, iters_per_sync=8)
        if r["rc"] != 0:
            continue
        ok += 1
        _validate(oracle_lib, prob, r["states"], goals, r["U"])
    assert ok >= 2


def test_single_goal_sequence_equals_plan():
    from paper_2609_30533_amd.lib import Problem, plan_sequence
    torch_cuda()
    prob = scenes.disc2d(0)
    prob.params.batch = 512
    r1 = plan_sequence(prob, prob.q_goal[None], max_iters=64, iters_per_sync=8)
    r2 = Problem(prob).plan(max_iters=64, iters_per_sync=8)
    assert r1["rc"] == r2["rc"]
    if r2["rc"] == 0:
        assert r1["U"] == r2["U"] and np.array_equal(r1["states"], r2["states"])


def test_goal_sequences_batched(oracle_lib):
    """Goal sequences of many problems at once (leg i of every problem in one
    batch): every returned path is re-validated in absolute time against the
    unshifted scene, and with an iteration budget each problem's path equals
    the one st_plan_sequence finds for it alone (a batch member's trees equal
    the single run's, iteration for iteration)."""
    from paper_2609_30533_amd.lib import plan_sequence, plan_sequence_batch
    torch_cuda()
    probs, goal_lists = [], []
    for seed in range(8):
        prob = scenes.disc2d(seed)
        prob.params.batch = 256
        prob.params.cap_fwd, prob.params.cap_bwd = 1 << 15, 1 << 12
        probs.append(prob)
        goal_lists.append(_goals(prob, 2 + seed % 3, seed))
    banner("batched sequences: %d problems" % len(probs))
    res = plan_sequence_batch(probs, goal_lists, max_iters=200, iters_per_sync=8)
    ok = 0
    for k, (prob, goals, r) in enumerate(zip(probs, goal_lists, res)):
        single = plan_sequence(prob, goals, max_iters=200, iters_per_sync=8, problem_id=k)
        assert r["rc"] == single["rc"], (k, r["rc"], single["rc"])
        if r["rc"] != 0:
            continue
        ok += 1
        _validate(oracle_lib, prob, r["states"], goals, r["U"])
        assert np.array_equal(r["states"], single["states"]), k
        assert r["U"] == single["U"]
    banner("batched sequences: %d of %d solved" % (ok, len(probs)))
    assert ok >= 5
