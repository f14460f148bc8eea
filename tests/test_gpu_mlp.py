"""Parity of the proposal network's device kernels (forward, loss, backward,
Adam) with the FP64 reference, and of the learned sampler with the oracle.

The device rounds every GEMM operand to bfloat16 and accumulates in FP32; the
reference rounds the forward operands the same way and computes the rest in
FP64 (the backward GEMMs of the device also round the incoming gradient, the
reference does not).  Bounds: network outputs within a relative L2 error of
1e-3, per-row losses within 1e-4, each parameter gradient within a relative
L2 error of 1e-2, one Adam step within 1e-6 of the reference update applied to
the device gradients."""
import math

import numpy as np
import pytest

from oracle import mlp as ref
from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

ORDER = ["We", "be", "W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5"]


def _flat(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float32).reshape(-1) for k in ORDER])


def _unflat(v, like):
    out, o = {}, 0
    for k in ORDER:
        n = like[k].size
        out[k] = v[o:o + n].reshape(like[k].shape).astype(np.float64)
        o += n
    assert o == v.size
    return out


def _batch(M, O, K, seed):
    rng = np.random.default_rng(seed)
    core = scenes.f32(rng.uniform(-1, 1, size=(M, ref.CORE)))
    obs = scenes.f32(rng.uniform(-1, 1, size=(M, O, ref.ENC_IN)))
    mask = (rng.random((M, O)) < 0.7).astype(np.float64)
    mask[:, 0] = 1
    mask[M // 3] = 0            # a row without obstacles pools to zero
    y = scenes.f32(rng.uniform(-1, 1, size=(M, K, ref.N_DIM)))
    ymask = (rng.random((M, K)) < 0.85).astype(np.float64)
    ymask[:, 0] = 1
    ymask[M // 2] = 0           # a row without states keeps only the histogram term
    dmask = np.zeros((M, ref.N_DIM))
    for i in range(M):
        d = 2 + i % 6
        dmask[i, :d] = 1
        dmask[i, 7] = 1
    ubin = rng.integers(0, ref.N_BINS, size=M).astype(np.int32)
    return core, obs, mask, y, ymask, dmask, ubin


def _dev(*arrs):
    torch = torch_cuda()
    return [to_dev(a, torch.int32 if a.dtype == np.int32 else torch.float32) for a in arrs]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# M spans two 64-row tiles with a ragged tail; M*O rows for the encoder too;
# 1100 rows split the weight-gradient reductions (split-K) and the bias sums
@pytest.mark.parametrize("M,O,K,seed", [(70, 5, 6, 0), (1, 1, 1, 1), (200, 32, 16, 2), (1100, 12, 8, 4)])
def test_forward_loss_backward_match_reference(M, O, K, seed):
    from paper_2609_30533_amd.lib import Mlp
    torch = torch_cuda()
    banner("mlp M=%d O=%d K=%d" % (M, O, K))
    p = ref.init_params(seed)
    rng = np.random.default_rng(100 + seed)
    for k in p:  # non-zero biases so the bias paths are exercised
        if k.startswith("b"):
            p[k] = scenes.f32(rng.normal(size=p[k].shape) * 0.1).astype(np.float32)
    core, obs, mask, y, ymask, dmask, ubin = _batch(M, O, K, seed)
    net = Mlp(max(M, 8), max(O, 4))
    net.set_params(_flat(p))
    dc, do, dm, dy, dym, ddm, dub = _dev(core, obs, mask, y, ymask, dmask, ubin)
    z = net.forward(dc, do, dm)
    per = net.loss(dy, dym, ddm, dub)
    net.backward()
    torch.cuda.synchronize()
    z = z.cpu().numpy().astype(np.float64)
    per = per.cpu().numpy().astype(np.float64)
    g = _unflat(net.grads(), p)

    zr, cache = ref.forward(p, core, obs, mask)
    assert np.all(np.isfinite(z))
    assert _rel(z, zr) <= 1e-3, _rel(z, zr)
    assert np.max(np.abs(z - zr)) <= 1e-2 * max(1.0, np.max(np.abs(zr)))
    # the loss kernel on the device's own z
    for i in range(M):
        Li, _ = ref.loss(z[i:i + 1], y[i:i + 1], ymask[i:i + 1], dmask[i:i + 1], ubin[i:i + 1])
        assert abs(per[i] - Li) <= 1e-4 * max(1.0, abs(Li)), (i, per[i], Li)
    # gradients against the reference chain on the reference z
    _, dz = ref.loss(zr, y, ymask, dmask, ubin)
    gr = ref.backward(p, cache, dz)
    for k in ORDER:
        if np.linalg.norm(gr[k]) == 0:
            assert np.allclose(g[k], 0, atol=1e-6), k
            continue
        assert _rel(g[k], gr[k]) <= 1e-2, (k, _rel(g[k], gr[k]))


def test_adam_step_matches_reference():
    from paper_2609_30533_amd.lib import Mlp
    torch = torch_cuda()
    banner("mlp adam")
    M, O, K = 48, 6, 8
    p = ref.init_params(7)
    core, obs, mask, y, ymask, dmask, ubin = _batch(M, O, K, 7)
    net = Mlp(M, O)
    net.set_params(_flat(p))
    dc, do, dm, dy, dym, ddm, dub = _dev(core, obs, mask, y, ymask, dmask, ubin)
    pr = {k: v.astype(np.float64) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in pr.items()}
    v = {k: np.zeros_like(v) for k, v in pr.items()}
    for t in (1, 2, 3):
        net.forward(dc, do, dm)
        net.loss(dy, dym, ddm, dub)
        net.backward()
        torch.cuda.synchronize()
        g = _unflat(net.grads(), p)
        net.adam(1e-3)
        torch.cuda.synchronize()
        pr, m, v = ref.adam_step(pr, g, m, v, t, lr=1e-3)
        pr = {k: x.astype(np.float64) for k, x in pr.items()}
        pd = _unflat(net.get_params(), p)
        for k in ORDER:
            assert np.max(np.abs(pd[k] - pr[k])) <= 1e-6 * max(1.0, np.max(np.abs(pr[k]))), (t, k)
        pr = pd  # continue from the device weights


def test_training_reduces_loss_on_a_fixed_batch():
    from paper_2609_30533_amd.lib import Mlp
    torch = torch_cuda()
    banner("mlp train")
    M, O, K = 64, 8, 16
    p = ref.init_params(3)
    core, obs, mask, y, ymask, dmask, ubin = _batch(M, O, K, 3)
    net = Mlp(M, O)
    net.set_params(_flat(p))
    dc, do, dm, dy, dym, ddm, dub = _dev(core, obs, mask, y, ymask, dmask, ubin)
    losses = []
    for _ in range(60):
        net.forward(dc, do, dm)
        per = net.loss(dy, dym, ddm, dub)
        losses.append(float(per.mean()))
        net.backward()
        net.adam(2e-3)
    torch.cuda.synchronize()
    assert all(math.isfinite(x) for x in losses)
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])


def test_bad_shapes_are_errors():
    from paper_2609_30533_amd.lib import Mlp, StError
    torch = torch_cuda()
    net = Mlp(8, 4)
    a = torch.zeros(16, ref.CORE, device="cuda")
    b = torch.zeros(16, 4, ref.ENC_IN, device="cuda")
    c = torch.ones(16, 4, device="cuda")
    with pytest.raises(StError):
        net.forward(a, b, c)          # 16 rows > capacity 8
    with pytest.raises(StError):
        net.adam(0.0)


def _proposal_z(prob, rng, spread=0.15):
    """A hand-made network output: components centred along the straight
    segment from start to goal, times along the arrival range."""
    z = np.zeros(ref.N_OUT)
    z[:ref.N_COMP] = rng.normal(size=ref.N_COMP)
    for c in range(ref.N_COMP):
        a = (c + 0.5) / ref.N_COMP
        q = (1 - a) * prob.q_start + a * prob.q_goal
        mu = np.zeros(ref.N_DIM)
        mu[:prob.d] = q / math.pi
        mu[7] = (prob.t_min + a * (prob.t_max - prob.t_min) * 0.5) / 60.0
        z[ref.N_COMP + c * ref.N_DIM:ref.N_COMP + (c + 1) * ref.N_DIM] = mu
        ls = np.full(ref.N_DIM, math.log(spread))
        ls[7] = math.log(0.5 * (prob.t_max - prob.t_min) / 60.0)
        off = ref.N_COMP + ref.N_COMP * ref.N_DIM
        z[off + c * ref.N_DIM:off + (c + 1) * ref.N_DIM] = ls
    z[-ref.N_BINS:] = rng.normal(size=ref.N_BINS)
    return scenes.f32(z)


LEARNED = [
    ("disc2d-ir", lambda: scenes.disc2d(1)),
    ("arm6-ir", lambda: scenes.arm6(2)),
    ("arm7-rr", lambda: scenes.arm7rr(2, n_obs=16)),
]


@pytest.mark.parametrize("name,make", LEARNED, ids=[p[0] for p in LEARNED])
def test_learned_sampling_matches_oracle(oracle_lib, name, make):
    from paper_2609_30533_amd.lib import Problem
    torch = torch_cuda()
    prob = make()
    prob.params.batch = 1024
    prob.params.cap_fwd = 1 << 14
    prob.params.cap_bwd = 1 << 11
    banner("learned sample %s" % name)
    z = _proposal_z(prob, np.random.default_rng(5))
    gp = Problem(prob)
    gp.set_proposal(to_dev(z, torch.float32), 0.5)
    op = oracle_lib.Planner(prob)
    op.set_proposal(z, 0.5)
    B = prob.params.batch
    n_learned = 0
    for it in (0, 3):
        s = {k: v.cpu().numpy() for k, v in gp.sample(it).items()}
        r = op.sample(it, B)
        assert np.array_equal(s["dir"], r["dir"])
        lf = (r["flags"] & 4) != 0
        assert np.array_equal((s["flags"] & 4) != 0, lf)
        n_learned += int(lf.sum())
        same = s["flags"] == r["flags"]
        # a differing flag may only come from a draw at a decision boundary
        assert (~same).sum() <= 0.01 * B, (~same).sum()
        both = same & ((r["flags"] & 1) == 0)
        np.testing.assert_allclose(s["qr"][:, both], r["qr"][:, both], rtol=1e-5, atol=1e-5)
        np.testing.assert_allclose(s["T"][both], r["T"][both], rtol=1e-5, atol=1e-5)
        assert np.array_equal(s["grp"][both], r["grp"][both])
        np.testing.assert_allclose(s["tr"][both], r["tr"][both], rtol=1e-5, atol=1e-4)
    # about half of the draws come from the network
    assert 0.4 * 2 * B <= n_learned <= 0.6 * 2 * B
    # switching it off restores the plain sampler
    gp.set_proposal(None)
    op.set_proposal(None, 0.0)
    s = {k: v.cpu().numpy() for k, v in gp.sample(1).items()}
    r = op.sample(1, B)
    assert not np.any(s["flags"] & 4)
    np.testing.assert_allclose(s["qr"], r["qr"], rtol=1e-6, atol=1e-6)
