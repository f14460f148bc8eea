"""Host-side pieces of the benchmark (no GPU): the algorithmic cost per
space-time state that the edge-check roofline divides by, counted by hand
from the per-term costs (forward kinematics 69 per joint, sphere centres 18
each, obstacle centres 7 each, sphere pairs 8 each; static terms 63 per
link pair + 18 per sphere of the upper link + 8 per sphere pair, 26 per
sphere and box), and the bootstrap interval's direction."""
import numpy as np

import bench
from paper_2609_30533_amd import scenes


def test_flops_per_state_arm6():
    # 6 joints, 40 spheres, 16 obstacles: 6*69 + 40*18 + 16*7 + 40*16*8
    assert bench.flops_per_state(scenes.arm6(0)) == 414 + 720 + 112 + 5120 == 6366


def test_flops_per_state_arm7_recycling():
    # 7 joints, 60 spheres, 32 obstacles
    assert bench.flops_per_state(scenes.arm7rr(0)) == 7 * 69 + 60 * 18 + 32 * 7 + 60 * 32 * 8 == 17147


def test_flops_per_state_disc():
    # a translating disc: 3 for the state, 3 for its one sphere, then the
    # obstacle centres and pairs of its 8 discs
    assert bench.flops_per_state(scenes.disc2d(0)) == 3 + 3 + 8 * 7 + 8 * 8 == 126


def test_flops_per_state_static_terms():
    p = scenes.arm6static(0)
    links = np.asarray(p.sphere_link)
    extra = 0
    for la, lb in {tuple(q) for q in np.asarray(p.self_pairs).tolist()}:
        na, nb = int((links == la).sum()), int((links == lb).sum())
        if na and nb:
            extra += 63 + 18 * nb + 8 * na * nb
    extra += 26 * p.n_spheres * len(p.boxes)
    assert bench.flops_per_state(p) == 6366 + extra == 12826


def test_bootstrap_interval_direction():
    # b is a everywhere plus 1 ms: the interval of median(b) - median(a) is [1, 1]
    a = np.linspace(0.1, 5.0, 50)
    r = bench._bootstrap_median_diff(a, a + 1.0)
    assert abs(r["diff_ms"][0] - 1.0) < 1e-9 and abs(r["diff_ms"][1] - 1.0) < 1e-9
