"""FP64 reference of the learned proposal network (test infrastructure only).

The network is the learned (q, t) and arrival-time proposal of the build (not
part of the paper): a shared per-obstacle encoder, max-pooled over obstacles,
followed by four dense GELU layers of width 256 and two heads, an 8-component
diagonal Gaussian mixture over the normalised space-time state and a 32-bin
histogram over the arrival range.  The device keeps weights and every layer
input in bfloat16 and accumulates in FP32; this reference rounds the same
quantities to bfloat16 and computes everything else in FP64, so the two differ
only by accumulation order and FP32 rounding.

Shapes (all row-major, one row per problem or per example):
  obstacle rows  obs  [M, O, 65]  (16 waypoints x (t, x, y, z), radius)
  core input     core [M, 16]     (q_s, q_g padded to 7, t_min, t_max)
  encoder        We [65, 64], be [64]           phi = gelu(obs We + be), pooled = max_o phi
  trunk          x0 = [core, pooled, 0-pad] (96)
                 W1 [96, 256], W2..W4 [256, 256] h_l = gelu(h_{l-1} W_l + b_l)
  head           W5 [256, 168], b5 [168]         z = h4 W5 + b5
  z[:, 0:8] mixture logits, z[:, 8:72] means (8 x 8), z[:, 72:136] log std
  (8 x 8), z[:, 136:168] histogram logits.
"""
from __future__ import annotations

import math

import numpy as np

N_COMP = 8          # mixture components
N_DIM = 8           # padded (q, t) dimensions: 7 joints + time
N_BINS = 32         # arrival-time histogram bins
ENC_IN = 65         # 16 waypoints x 4 + radius
ENC_OUT = 64
CORE = 16           # q_s (7), q_g (7), t_min, t_max
D_IN = 96           # CORE + ENC_OUT padded to a multiple of 32
WIDTH = 256
N_OUT = N_COMP * (1 + 2 * N_DIM) + N_BINS   # 168
T_SCALE = 60.0      # seconds
Q_SCALE = math.pi   # radians (box half-width of the arms)

LAYER_SHAPES = [("We", (ENC_IN, ENC_OUT)), ("W1", (D_IN, WIDTH)), ("W2", (WIDTH, WIDTH)), ("W3", (WIDTH, WIDTH)),
                ("W4", (WIDTH, WIDTH)), ("W5", (WIDTH, N_OUT))]


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    out = (u.astype(np.uint32)).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def gelu(x):
    """Exact GELU, x Phi(x) with the Gaussian CDF written through erf."""
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(seed=0):
    """FP32 master weights: He-style normal init, zero biases (biases FP32)."""
    rng = np.random.default_rng([0x31337, seed])
    p = {}
    for name, (fi, fo) in LAYER_SHAPES:
        p[name] = (rng.normal(size=(fi, fo)) * math.sqrt(2.0 / fi)).astype(np.float32)
        p["b" + name[1:]] = np.zeros(fo, dtype=np.float32)
    p["W5"] *= 0.1
    return p


def forward(p, core, obs, mask):
    """core [M,16], obs [M,O,65], mask [M,O] (1 = real obstacle).  Returns z
    [M,168] and the cache for the backward pass."""
    M, O, _ = obs.shape
    c = {}
    xo = bf16(obs.reshape(M * O, ENC_IN))
    pre_e = xo @ bf16(p["We"]).astype(np.float64) + p["be"].astype(np.float64)
    phi = gelu(pre_e).reshape(M, O, ENC_OUT)
    phi_m = np.where(mask[:, :, None] > 0, phi, -np.inf)
    arg = np.argmax(phi_m, axis=1)                # first maximum on ties
    pooled = np.take_along_axis(phi_m, arg[:, None, :], axis=1)[:, 0, :]
    pooled = np.where(np.isfinite(pooled), pooled, 0.0)
    x0 = np.zeros((M, D_IN))
    x0[:, :CORE] = core
    x0[:, CORE:CORE + ENC_OUT] = pooled
    c.update(xo=xo, pre_e=pre_e, arg=arg, mask=mask, M=M, O=O)
    h = x0
    for l in range(1, 5):
        xin = bf16(h)
        pre = xin @ bf16(p["W%d" % l]) + p["b%d" % l].astype(np.float64)
        c["x%d" % l] = xin
        c["pre%d" % l] = pre
        h = gelu(pre)
    xin = bf16(h)
    z = xin @ bf16(p["W5"]) + p["b5"].astype(np.float64)
    c["x5"] = xin
    return z, c


def split_head(z):
    M = z.shape[0]
    logit = z[:, 0:N_COMP]
    mu = z[:, N_COMP:N_COMP + N_COMP * N_DIM].reshape(M, N_COMP, N_DIM)
    ls = z[:, N_COMP + N_COMP * N_DIM:N_COMP * (1 + 2 * N_DIM)].reshape(M, N_COMP, N_DIM)
    hist = z[:, N_COMP * (1 + 2 * N_DIM):]
    return logit, mu, ls, hist


def _logsumexp(a, axis):
    m = np.max(a, axis=axis, keepdims=True)
    return (m + np.log(np.sum(np.exp(a - m), axis=axis, keepdims=True))).squeeze(axis)


def loss(z, y, ymask, dmask, ubin):
    """Mixture NLL of the path states plus the arrival-bin cross-entropy.

    y [M,K,8] normalised states along each path, ymask [M,K] (1 = real state),
    dmask [M,8] (1 = dimension in use: the robot's joints and time),
    ubin [M] arrival bin.  Loss = mean over examples of
      (sum_k ymask NLL(y_k)) / (sum_k ymask) + CE(hist, ubin).
    Returns (loss, dz [M,168])."""
    M, K, D = y.shape
    logit, mu, ls, hist = split_head(z)
    logw = logit - _logsumexp(logit, 1)[:, None]                      # [M, C]
    diff = (y[:, :, None, :] - mu[:, None, :, :]) * np.exp(-ls)[:, None, :, :]   # [M,K,C,D]
    logn = (-0.5 * diff ** 2 - ls[:, None, :, :] - 0.5 * math.log(2 * math.pi)) * dmask[:, None, None, :]
    lj = logw[:, None, :] + logn.sum(axis=3)                           # [M,K,C]
    lp = _logsumexp(lj, 2)                                              # [M,K]
    cnt = np.maximum(ymask.sum(axis=1), 1.0)
    nll = -(lp * ymask).sum(axis=1) / cnt
    loghist = hist - _logsumexp(hist, 1)[:, None]
    ce = -loghist[np.arange(M), ubin]
    L = float(np.mean(nll + ce))
    # gradients
    r = np.exp(lj - lp[:, :, None]) * (ymask / cnt[:, None])[:, :, None]   # responsibilities x weight
    dlogit = -(r.sum(axis=1) - np.exp(logw) * r.sum(axis=(1, 2))[:, None])
    dmu = -(r[:, :, :, None] * diff * np.exp(-ls)[:, None, :, :] * dmask[:, None, None, :]).sum(axis=1)
    dls = -(r[:, :, :, None] * (diff ** 2 - 1.0) * dmask[:, None, None, :]).sum(axis=1)
    dhist = np.exp(loghist)
    dhist[np.arange(M), ubin] -= 1.0
    dz = np.concatenate([dlogit, dmu.reshape(M, -1), dls.reshape(M, -1), dhist], axis=1) / M
    return L, dz


def backward(p, c, dz):
    """Gradients of the loss with respect to the FP32 master parameters (the
    straight-through convention: the bfloat16 rounding of the weights and of
    the layer inputs is treated as the identity)."""
    g = {}
    g["W5"] = c["x5"].T @ dz
    g["b5"] = dz.sum(axis=0)
    dh = dz @ bf16(p["W5"]).T
    for l in range(4, 0, -1):
        dpre = dh * gelu_grad(c["pre%d" % l])
        g["W%d" % l] = c["x%d" % l].T @ dpre
        g["b%d" % l] = dpre.sum(axis=0)
        dh = dpre @ bf16(p["W%d" % l]).T
    dpool = dh[:, CORE:CORE + ENC_OUT]
    M, O = c["M"], c["O"]
    dphi = np.zeros((M, O, ENC_OUT))
    rows = np.arange(M)[:, None]
    cols = np.arange(ENC_OUT)[None, :]
    dphi[rows, c["arg"], cols] = dpool
    dphi = dphi * (c["mask"][:, :, None] > 0)
    dpre_e = dphi.reshape(M * O, ENC_OUT) * gelu_grad(c["pre_e"])
    g["We"] = c["xo"].T @ dpre_e
    g["be"] = dpre_e.sum(axis=0)
    return g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the FP32 master parameters (Kingma and Ba, 2015)."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = (p[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return p, m, v
