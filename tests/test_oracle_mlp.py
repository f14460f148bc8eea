"""Pins for the FP64 proposal-network reference (CPU only): central finite
differences of the loss through the whole network, the one-component mixture
against the textbook Gaussian negative log-likelihood, the histogram term
against the textbook cross-entropy, bfloat16 rounding against known values."""
import math

import numpy as np

from oracle import mlp


def _batch(M=3, O=5, K=4, seed=0):
    rng = np.random.default_rng(seed)
    core = rng.uniform(-1, 1, size=(M, mlp.CORE))
    obs = rng.uniform(-1, 1, size=(M, O, mlp.ENC_IN))
    mask = (rng.random((M, O)) < 0.8).astype(float)
    mask[:, 0] = 1
    y = rng.uniform(-1, 1, size=(M, K, mlp.N_DIM))
    ymask = (rng.random((M, K)) < 0.9).astype(float)
    ymask[:, 0] = 1
    dmask = np.zeros((M, mlp.N_DIM))
    dmask[:, :6] = 1
    dmask[:, 7] = 1
    ubin = rng.integers(0, mlp.N_BINS, size=M)
    return core, obs, mask, y, ymask, dmask, ubin


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.00390625, 1.005859375, -3.1415926, 1e-3, 65504.0])
    r = mlp.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0            # halfway between 1 and 1 + 2^-7: ties to even
    assert r[2] == 1.0078125      # above the half: rounds up
    assert abs(r[3] + 3.140625) < 1e-12
    assert abs(r[4] - 0.00099945068359375) < 1e-15
    # idempotent
    assert np.array_equal(mlp.bf16(r), r)


def test_single_component_is_gaussian_nll():
    M, K = 2, 3
    rng = np.random.default_rng(1)
    z = np.zeros((M, mlp.N_OUT))
    z[:, 0] = 0.0
    z[:, 1:mlp.N_COMP] = -1e9          # all weight on component 0
    mu = rng.normal(size=(M, mlp.N_DIM))
    ls = rng.normal(size=(M, mlp.N_DIM)) * 0.3
    z[:, mlp.N_COMP:mlp.N_COMP + mlp.N_DIM] = mu
    off = mlp.N_COMP + mlp.N_COMP * mlp.N_DIM
    z[:, off:off + mlp.N_DIM] = ls
    y = rng.normal(size=(M, K, mlp.N_DIM))
    ymask = np.ones((M, K))
    dmask = np.ones((M, mlp.N_DIM))
    ubin = np.zeros(M, dtype=int)
    L, _ = mlp.loss(z, y, ymask, dmask, ubin)
    # textbook: -log N(y; mu, diag(sigma^2)) averaged over states, plus -log(1/32)
    nll = 0.0
    for i in range(M):
        s = 0.0
        for k in range(K):
            sig = np.exp(ls[i])
            s += np.sum(0.5 * ((y[i, k] - mu[i]) / sig) ** 2 + np.log(sig) + 0.5 * math.log(2 * math.pi))
        nll += s / K + math.log(mlp.N_BINS)
    assert abs(L - nll / M) < 1e-9


def test_histogram_term_is_cross_entropy():
    M = 4
    rng = np.random.default_rng(2)
    z = np.zeros((M, mlp.N_OUT))
    h = rng.normal(size=(M, mlp.N_BINS))
    z[:, -mlp.N_BINS:] = h
    y = np.zeros((M, 1, mlp.N_DIM))
    ymask = np.zeros((M, 1))           # no states: the mixture term vanishes
    dmask = np.ones((M, mlp.N_DIM))
    ubin = rng.integers(0, mlp.N_BINS, size=M)
    L, dz = mlp.loss(z, y, ymask, dmask, ubin)
    ce = np.mean([-(h[i, ubin[i]] - np.log(np.exp(h[i]).sum())) for i in range(M)])
    assert abs(L - ce) < 1e-12
    sm = np.exp(h) / np.exp(h).sum(axis=1, keepdims=True)
    sm[np.arange(M), ubin] -= 1
    assert np.allclose(dz[:, -mlp.N_BINS:], sm / M)


def test_loss_gradient_finite_differences():
    core, obs, mask, y, ymask, dmask, ubin = _batch()
    rng = np.random.default_rng(3)
    z = rng.normal(size=(core.shape[0], mlp.N_OUT)) * 0.5
    L, dz = mlp.loss(z, y, ymask, dmask, ubin)
    eps = 1e-6
    for _ in range(40):
        i, j = rng.integers(0, z.shape[0]), rng.integers(0, mlp.N_OUT)
        zp, zm = z.copy(), z.copy()
        zp[i, j] += eps
        zm[i, j] -= eps
        num = (mlp.loss(zp, y, ymask, dmask, ubin)[0] - mlp.loss(zm, y, ymask, dmask, ubin)[0]) / (2 * eps)
        assert abs(num - dz[i, j]) <= 1e-6 * max(1.0, abs(num)) + 1e-8, (i, j, num, dz[i, j])


def test_network_gradient_finite_differences():
    """Through the whole network with the bfloat16 rounding switched off
    (rounding is piecewise constant, the backward pass treats it as identity)."""
    core, obs, mask, y, ymask, dmask, ubin = _batch(M=2, O=4, K=3, seed=4)
    p = mlp.init_params(1)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    saved = mlp.bf16
    mlp.bf16 = lambda x: np.asarray(x, dtype=np.float64)
    try:
        z, c = mlp.forward(p, core, obs, mask)
        L, dz = mlp.loss(z, y, ymask, dmask, ubin)
        g = mlp.backward(p, c, dz)
        rng = np.random.default_rng(5)
        eps = 1e-6
        for name in ["We", "be", "W1", "b1", "W3", "W5", "b5"]:
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in p[name].shape)
                old = p[name][idx]
                p[name][idx] = old + eps
                Lp = mlp.loss(mlp.forward(p, core, obs, mask)[0], y, ymask, dmask, ubin)[0]
                p[name][idx] = old - eps
                Lm = mlp.loss(mlp.forward(p, core, obs, mask)[0], y, ymask, dmask, ubin)[0]
                p[name][idx] = old
                num = (Lp - Lm) / (2 * eps)
                assert abs(num - g[name][idx]) <= 1e-6 * max(1.0, abs(num)) + 1e-7, (name, idx, num, g[name][idx])
    finally:
        mlp.bf16 = saved


def test_gelu_matches_definition():
    x = np.linspace(-6, 6, 101)
    from scipy.stats import norm
    assert np.allclose(mlp.gelu(x), x * norm.cdf(x), atol=1e-14)
    h = 1e-6
    assert np.allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), atol=1e-8)
