"""Parity of st_nearest with the FP64 oracle on imported trees.

Index results must match exactly unless the oracle flags the query as
fragile (a runner-up within a relative 1e-5, or a near-best node within 1e-5
of the speed cone); then the device's choice must still be within 1e-5 of the
oracle's best.  Distances agree within a relative 1e-5."""
import math

import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _random_state(prob, n_fwd, n_bwd, seed, U):
    """Fill the forward pool and every backward pool with random nodes."""
    rng = np.random.default_rng(seed)
    p = prob.params
    N = p.n_groups
    total = p.cap_fwd + N * p.cap_bwd
    d = prob.d
    x = np.zeros((total, d + 1), dtype=np.float32)
    parent = np.full(total, -1, dtype=np.int32)
    cost = np.zeros(total, dtype=np.float32)
    rootT = np.zeros(total, dtype=np.float32)
    counts = np.zeros(1 + N, dtype=np.int64)
    q, t, _ = scenes.synthetic_tree(prob, n_fwd, seed=seed)
    x[:n_fwd, :d], x[:n_fwd, d] = q, t
    counts[0] = n_fwd
    for g in range(N):
        base = p.cap_fwd + g * p.cap_bwd
        n = int(rng.integers(0, n_bwd + 1))
        q, t, _ = scenes.synthetic_tree(prob, max(n, 1), seed=seed * 100 + g)
        x[base:base + n, :d], x[base:base + n, d] = q[:n], t[:n]
        # a few trees per group, root times on either side of U
        roots = scenes.f32(rng.uniform(prob.t_min, prob.t_max, size=4))
        rootT[base:base + n] = roots[rng.integers(0, 4, size=n)]
        counts[1 + g] = n
    return dict(counts=counts, x=x, parent=parent, cost=cost, rootT=rootT, U=U)


def _oracle_nearest(o, prob, st, set_id, metric, sigma, xq):
    p = prob.params
    N = p.n_groups
    pools = [0] if set_id == -1 else (list(range(1, N + 1)) if set_id == -2 else [1 + set_id])
    idxs, rows = [], []
    for pool in pools:
        base = 0 if pool == 0 else p.cap_fwd + (pool - 1) * p.cap_bwd
        for i in range(base, base + int(st["counts"][pool])):
            if pool > 0 and prob.params.variant == 0 and not (st["rootT"][i] < st["U"]):
                continue
            idxs.append(i)
            rows.append(st["x"][i])
    idxs = np.array(idxs, dtype=np.int64)
    nodes = np.array(rows, dtype=np.float64).reshape(-1, prob.d + 1)
    out = []
    for x in xq:
        k, dist, amb = o.nearest(nodes, x.astype(np.float64), sigma=sigma, metric=metric)
        out.append((int(idxs[k]) if k >= 0 else -1, dist, amb))
    return out, nodes, idxs


CASES = [
    ("arm6-fwd-rho", scenes.arm6, -1, 0, 1),
    ("arm6-group-rho", scenes.arm6, 3, 0, -1),
    ("arm6-allbwd-rho", scenes.arm6, -2, 0, -1),
    ("disc-fwd-rho", scenes.disc2d, -1, 0, 1),
    ("arm7-fwd-config", scenes.arm7rr, -1, 1, 1),
    ("arm7-slot-config", scenes.arm7rr, 5, 1, -1),
]


@pytest.mark.parametrize("name,maker,set_id,metric,sigma", CASES, ids=[c[0] for c in CASES])
def test_nearest_matches_oracle(oracle_lib, name, maker, set_id, metric, sigma):
    from paper_2609_30533_amd.lib import Problem
    prob = maker(2)
    prob.params.cap_fwd = 1 << 14
    prob.params.cap_bwd = 1 << 11
    if prob.params.n_groups > 16:
        prob.params.n_groups = 16
    banner("nearest %s" % name)
    U = float(scenes.f32(0.5 * (prob.t_min + prob.t_max)))
    st = _random_state(prob, 12000 + 17, 1500, seed=3, U=U)
    gp = Problem(prob)
    slots = None
    if prob.params.variant == 1:
        N = prob.params.n_groups
        slots = (np.full(N, 5.0), np.ones(N, np.int32), np.zeros(N, np.uint32), np.zeros(N, np.int64))
    gp.import_state(st["counts"], st["x"], st["parent"], st["cost"], st["rootT"], U, math.inf, -1, -1, 0, slots)
    xq = scenes.synthetic_states(prob, 1024 + 9, seed=4)
    idx, dist = gp.nearest(to_dev(xq), set_id=set_id, metric=metric, sigma=sigma)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    o = oracle_lib.Oracle(prob)
    ref, nodes, idxs = _oracle_nearest(o, prob, st, set_id, metric, sigma, xq)
    n_amb = 0
    found = 0
    for i, (ri, rd, amb) in enumerate(ref):
        if ri >= 0:
            found += 1
        if amb:
            n_amb += 1
            # any near-best choice is acceptable
            if idx[i] >= 0 and ri >= 0:
                y = st["x"][idx[i]].astype(np.float64)
                r = o.rho(sigma, y, xq[i].astype(np.float64)) if metric == 0 else \
                    np.linalg.norm(y[:prob.d] - xq[i, :prob.d])
                assert r <= rd * (1 + 1e-5) + 1e-6
            continue
        assert idx[i] == ri, (i, idx[i], ri)
        if ri >= 0:
            assert abs(dist[i] - rd) <= 1e-5 * max(rd, 1e-6) + 1e-6
        else:
            assert math.isinf(dist[i])
    assert n_amb < 0.10 * len(ref)
    assert found > 0.3 * len(ref)


def test_nearest_ties_and_empty(oracle_lib):
    from paper_2609_30533_amd.lib import Problem
    prob = scenes.disc2d(0)
    prob.params.cap_fwd = 256
    prob.params.cap_bwd = 64
    gp = Problem(prob)
    N = prob.params.n_groups
    total = 256 + N * 64
    x = np.zeros((total, 3), dtype=np.float32)
    x[:5] = [[0.5, 0.5, 1.0], [0.2, 0.2, 0.0], [0.5, 0.5, 1.0], [0.5, 0.5, 1.0], [0.9, 0.9, 5.0]]
    counts = np.zeros(1 + N, dtype=np.int64)
    counts[0] = 5
    z = np.zeros(total, dtype=np.float32)
    gp.import_state(counts, x, np.full(total, -1, np.int32), z, z, math.inf, math.inf, -1, -1, 0)
    q = np.array([[0.5, 0.5, 2.0], [0.5, 0.5, 0.5]], dtype=np.float32)
    idx, dist = gp.nearest(to_dev(q), set_id=-1, metric=0, sigma=1)
    idx = idx.cpu().numpy()
    assert idx[0] == 0            # three identical nodes: lowest index
    assert idx[1] == 1            # only the node at t = 0 precedes t = 0.5 ... and is reachable
    # an empty backward group has no admissible node
    idx, dist = gp.nearest(to_dev(q), set_id=2, metric=0, sigma=-1)
    assert (idx.cpu().numpy() == -1).all() and np.isinf(dist.cpu().numpy()).all()
    # M = 0 is a no-op
    torch = torch_cuda()
    gp.nearest(torch.zeros(0, 3, device="cuda"))
