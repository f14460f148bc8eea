"""Parity of st_check_states / st_check_edges with the FP64 oracle.

Index and boolean results must match bit for bit unless some checked state
is within 1e-4 of a contact (|margin| <= 1e-4) or the state count n is
ambiguous (max(D, v dt)/h within 1e-6 of an integer)."""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

MARGIN = 1e-4


def _exempt(res):
    nr = res["n_real"]
    amb_n = np.abs(nr - np.round(nr)) <= 1e-6 * np.maximum(nr, 1.0)
    return (res["margin"] <= MARGIN) | amb_n


def _generic_times(prob):
    """Same obstacles, but each obstacle with its own waypoint times."""
    rng = np.random.default_rng(9)
    wp = prob.wp.copy()
    for o in range(prob.n_obs):
        n = prob.n_wp[o]
        inner = np.sort(rng.uniform(0, prob.t_max, size=n - 2))
        wp[o, 1:n - 1, 0] = inner
    prob.wp = scenes.f32(wp)
    return prob


CASES = [
    ("disc2d", lambda: scenes.disc2d(3), 4096 + 37),
    ("arm6", lambda: scenes.arm6(3), 1536 + 29),
    ("arm7rr", lambda: scenes.arm7rr(3), 768 + 13),
    ("arm6-generic-times", lambda: _generic_times(scenes.arm6(4, n_wp=5)), 768 + 5),
    ("arm6-5obs", lambda: scenes.arm6(5, n_obs=5), 1024 + 3),
    ("mixed-64obs", lambda: scenes.arm6(6, n_obs=64, n_wp=4), 512 + 1),
]


@pytest.mark.parametrize("name,make,E", CASES, ids=[c[0] for c in CASES])
def test_edges_match_oracle(oracle_lib, name, make, E):
    from paper_2609_30533_amd.lib import Problem
    prob = make()
    banner("edges %s E=%d" % (name, E))
    xa, xb = scenes.synthetic_edges(prob, E, seed=21, bridge_mix=True)
    orc = oracle_lib.Oracle(prob).check_edges(xa, xb)
    gp = Problem(prob)
    free, fh = gp.check_edges(to_dev(xa), to_dev(xb), first_hit=True)
    free2, _ = gp.check_edges(to_dev(xa), to_dev(xb), first_hit=False)
    torch = torch_cuda()
    torch.cuda.synchronize()
    free, fh, free2 = free.cpu().numpy(), fh.cpu().numpy(), free2.cpu().numpy()
    ex = _exempt(orc)
    ok = ~ex
    assert ex.mean() < 0.05, ex.mean()
    assert np.array_equal(free[ok], orc["free"][ok]), np.where(free[ok] != orc["free"][ok])
    assert np.array_equal(fh[ok], orc["first_hit"][ok])
    assert np.array_equal(free2[ok], orc["free"][ok])
    # both outcomes occur
    assert 0.003 < orc["free"].mean() < 0.997


def test_edges_reversed_endpoints_identical(oracle_lib):
    from paper_2609_30533_amd.lib import Problem
    prob = scenes.arm6(8)
    xa, xb = scenes.synthetic_edges(prob, 2000, seed=5)
    gp = Problem(prob)
    f1, h1 = gp.check_edges(to_dev(xa), to_dev(xb))
    f2, h2 = gp.check_edges(to_dev(xb), to_dev(xa))
    assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
    assert np.array_equal(h1.cpu().numpy(), h2.cpu().numpy())


@pytest.mark.parametrize("maker", [lambda: scenes.arm6(3), lambda: scenes.arm7rr(2)], ids=["arm6", "arm7rr"])
def test_launch_shapes_do_not_change_results(oracle_lib, maker):
    """Obstacle tile, lanes per chunk and lanes per state change the schedule
    only: free flags and least colliding indices are identical, and agree
    with the oracle wherever it does not exempt the decision."""
    from paper_2609_30533_amd.lib import Problem
    prob = maker()
    banner("launch shapes %s" % prob.name)
    xa, xb = scenes.synthetic_edges(prob, 3000, seed=11, bridge_mix=True)
    gp = Problem(prob)
    da, db = to_dev(xa), to_dev(xb)
    ref = None
    for ot in (8, 16):
        for lanes in (16, 32, 64):
            for split in (1, 2, 4):
                gp.set_tuning(obstacle_tile=ot, lanes_check=lanes)
                gp.set_state_split(check=split)
                f, h = gp.check_edges(da, db)
                cur = (f.cpu().numpy(), h.cpu().numpy())
                if ref is None:
                    ref = cur
                    continue
                assert np.array_equal(cur[0], ref[0]), (ot, lanes, split)
                assert np.array_equal(cur[1], ref[1]), (ot, lanes, split)
    res = oracle_lib.Oracle(prob).check_edges(xa, xb)
    ok = ~_exempt(res)
    assert np.array_equal(ref[0][ok].astype(bool), res["free"][ok].astype(bool))


@pytest.mark.parametrize("maker", [lambda: scenes.disc2d(4), lambda: scenes.arm6(3, n_obs=5)], ids=["disc2d", "arm6-5obs"])
def test_forced_obstacle_tile_pads_without_changing_results(maker):
    """A problem created with a forced obstacle tile (its obstacles padded
    with far, zero-radius ones) decides every state and edge as the same
    problem with the automatic tile, and plans the same trees."""
    from paper_2609_30533_amd.lib import Problem
    torch = torch_cuda()
    base = maker()
    banner("forced obstacle tile %s" % base.name)
    xa, xb = scenes.synthetic_edges(base, 3000, seed=13, bridge_mix=True)
    da, db = to_dev(xa), to_dev(xb)
    ref = None
    for tile in (0, 4, 8, 16):
        prob = maker()
        prob.params.batch = 256
        prob.params.obstacle_tile = tile
        gp = Problem(prob)
        f, h = gp.check_edges(da, db)
        gp.iterate(6)
        torch.cuda.synchronize()
        ex = gp.export()
        cur = (f.cpu().numpy(), h.cpu().numpy(), ex["counts"], gp.info()["obstacle_tile"])
        if tile:
            assert cur[3] == tile
        if ref is None:
            ref = cur
            continue
        assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), tile
        assert np.array_equal(cur[2], ref[2]), tile
        gp.close()


def test_edges_degenerate_and_long(oracle_lib):
    """Zero-length edges, pure waits, edges leaving the box or the horizon,
    and long bridges that span thousands of states."""
    from paper_2609_30533_amd.lib import Problem
    prob = scenes.arm6(9)
    rng = np.random.default_rng(1)
    rows_a, rows_b = [], []
    for _ in range(64):
        q = rng.uniform(-3, 3, 6)
        t = rng.uniform(0, 19)
        rows_a.append(np.r_[q, t]); rows_b.append(np.r_[q, t])                 # a single state
        rows_a.append(np.r_[q, t]); rows_b.append(np.r_[q, min(t + 1.0, 20)])  # waiting
        q2 = q.copy(); q2[0] = 3.3                                              # leaves the box
        rows_a.append(np.r_[q, t]); rows_b.append(np.r_[q2, t + 0.5])
        rows_a.append(np.r_[q, 19.9]); rows_b.append(np.r_[q, 20.5])            # leaves the horizon
        q3 = rng.uniform(-3, 3, 6)
        rows_a.append(np.r_[q, 0.5]); rows_b.append(np.r_[q3, 19.5])            # long bridge
    xa = np.array(rows_a, dtype=np.float32)
    xb = np.array(rows_b, dtype=np.float32)
    orc = oracle_lib.Oracle(prob).check_edges(xa, xb)
    assert orc["n"].max() > 1000
    gp = Problem(prob)
    free, fh = gp.check_edges(to_dev(xa), to_dev(xb))
    free, fh = free.cpu().numpy(), fh.cpu().numpy()
    ok = ~_exempt(orc)
    assert np.array_equal(free[ok], orc["free"][ok])
    assert np.array_equal(fh[ok], orc["first_hit"][ok])
    # empty batch is a no-op
    torch = torch_cuda()
    gp.check_edges(torch.zeros(0, 7, device="cuda"), torch.zeros(0, 7, device="cuda"))


@pytest.mark.parametrize("maker", [scenes.disc2d, scenes.arm6, scenes.arm7rr])
def test_states_match_oracle(oracle_lib, maker):
    from paper_2609_30533_amd.lib import Problem
    prob = maker(11)
    banner("states %s" % prob.name)
    x = scenes.synthetic_states(prob, 3000 + 7, seed=2)
    free_o, margin = oracle_lib.Oracle(prob).check_states(x)
    gp = Problem(prob)
    free = gp.check_states(to_dev(x)).cpu().numpy()
    ok = np.abs(margin) > MARGIN
    assert np.array_equal(free[ok], free_o[ok])


def test_goal_grid_matches_oracle(oracle_lib):
    from paper_2609_30533_amd.lib import Problem
    for maker in (scenes.disc2d, scenes.arm6, scenes.arm7rr):
        prob = maker(12)
        o = oracle_lib.Oracle(prob)
        k_lo, k_hi, free_o = o.goal_grid()
        gp = Problem(prob)
        inf = gp.info()
        assert (inf["k_lo"], inf["k_hi"]) == (k_lo, k_hi)
        free = gp.goal_free()
        xs = np.array([np.r_[prob.q_goal, k * prob.params.dt] for k in range(k_lo, k_hi + 1)])
        _, m = o.check_states(xs)
        ok = np.abs(m) > MARGIN
        assert np.array_equal(free[ok], free_o[ok])


def test_full_size_sampled(oracle_lib):
    """2^20 synthetic edges on the 6-DOF arm in the launch shape the benchmark
    times; 400 sampled outputs are checked one by one against the oracle."""
    from paper_2609_30533_amd.lib import Problem
    prob = scenes.arm6(0)
    E = 1 << 20
    banner("full-size edges E=%d" % E)
    xa, xb = scenes.synthetic_edges(prob, E, seed=99)
    gp = Problem(prob)
    free, fh = gp.check_edges(to_dev(xa), to_dev(xb), first_hit=True)
    free, fh = free.cpu().numpy(), fh.cpu().numpy()
    rng = np.random.default_rng(0)
    pick = rng.choice(E, 400, replace=False)
    orc = oracle_lib.Oracle(prob).check_edges(xa[pick], xb[pick])
    ok = ~_exempt(orc)
    assert np.array_equal(free[pick][ok], orc["free"][ok])
    assert np.array_equal(fh[pick][ok], orc["first_hit"][ok])
    assert 0.05 < free.mean() < 0.95


@pytest.mark.parametrize("piecewise", [False, True], ids=["constant-velocity", "piecewise"])
def test_continuous_check_matches_oracle(oracle_lib, piecewise):
    """The exact continuous check against the oracle's closed form: free flags
    bit-exact wherever the clearance is not within 1e-4 of contact, least
    clearance within 1e-5."""
    from paper_2609_30533_amd.lib import Problem
    from tests.test_oracle_geometry import _piecewise_disc
    prob = _piecewise_disc(8) if piecewise else scenes.disc2d(5)
    banner("continuous %s" % ("piecewise" if piecewise else "linear"))
    xa, xb = scenes.synthetic_edges(prob, 3000, seed=15, bridge_mix=True)
    gp = Problem(prob)
    f, dm = gp.check_edges_continuous(to_dev(xa), to_dev(xb))
    f, dm = f.cpu().numpy(), dm.cpu().numpy()
    o = oracle_lib.Oracle(prob)
    n_free = n_hit = 0
    for e in range(len(xa)):
        ok, m = o.edge_continuous_pw(xa[e].astype(np.float64), xb[e].astype(np.float64))
        assert abs(dm[e] - m) <= 1e-5 * max(1.0, abs(m)), (e, dm[e], m)
        if abs(m) > MARGIN:
            assert bool(f[e]) == ok, (e, f[e], ok, m)
            n_free += ok
            n_hit += not ok
    assert n_free > 200 and n_hit > 200


def test_continuous_check_rejects_arms():
    from paper_2609_30533_amd.lib import Problem, StError
    prob = scenes.arm6(1)
    gp = Problem(prob)
    x = to_dev(np.zeros((4, 7), dtype=np.float32))
    with pytest.raises(StError):
        gp.check_edges_continuous(x, x)
