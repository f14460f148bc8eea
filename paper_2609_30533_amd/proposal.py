"""The learned proposal: harvesting solution paths with the plain planner,
training the network on the device, and installing its output in problems.

Every arithmetic step runs in the library's kernels (planning, forward,
loss, backward and Adam passes of the network); this module only moves data:
it builds feature and target rows from problems and paths, batches them, and
keeps the weights on disk as a flat FP32 array (layout We, be, W1, b1, ...,
W5, b5 with every W row-major [in][out]).

Usage on a machine with the device::

    python -m paper_2609_30533_amd.proposal --paths 20000 --out weights.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import scenes
from .lib import Batch, Mlp, Problem, ST_MLP_OUTPUTS

O_MAX = 32          # obstacle rows per problem fed to the encoder
K_STATES = 16       # path states per training example
TRAIN_SEED0 = 1_000_000  # training problems use seeds from here on; evaluation seeds stay below


def harvest_problem(seed: int):
    """A training problem of the 6-DOF arm workload, drawn as the evaluation
    problems are (start and goal redrawn until the library finds the start
    free and some goal-grid time free), with a smaller sample count so that
    many of them share the device; None when no draw is accepted."""
    from .problems import eval_problem
    p, _ = eval_problem("arm6", seed, max_attempts=16)
    if p is None:
        return None
    p.params.batch = 512
    p.params.cap_fwd = 1 << 16
    p.params.cap_bwd = 1 << 13
    return p


def harvest(n_paths: int, per_batch: int = 128, max_ms: float = 2500.0, seed0: int = TRAIN_SEED0,
            log=print, time_limit_s: float = 1e9):
    """Plan batches of training problems until n_paths solution paths exist.
    Returns a list of (problem, path) with path a dict holding the states
    [n, d+1], arrival U and length C."""
    out = []
    seed = seed0
    t0 = time.time()
    while len(out) < n_paths and time.time() - t0 < time_limit_s:
        probs = [q for q in (harvest_problem(seed + i) for i in range(per_batch)) if q is not None]
        seed += per_batch
        if not probs:
            continue
        gps = [Problem(p, problem_id=i) for i, p in enumerate(probs)]
        b = Batch(gps)
        r = b.plan(max_ms=max_ms, stop_at_first=False)
        for p, gp, f in zip(probs, gps, r["first_iter"]):
            if f < 0:
                continue
            path = gp.path()
            if path["rc"] == 0 and path["states"] is not None and len(path["states"]) >= 2:
                out.append((p, path))
        b.close()
        for gp in gps:
            gp.close()
        log("[harvest] %d paths after %d problems (%.0f s)" % (len(out), seed - seed0, time.time() - t0))
    return out[:n_paths]


def make_dataset(pairs, o_max=O_MAX, k=K_STATES):
    """Feature and target arrays for a list of (problem, path dict)."""
    M = len(pairs)
    core = np.zeros((M, scenes.PROP_CORE), dtype=np.float32)
    obs = np.zeros((M, o_max, scenes.PROP_ENC_IN), dtype=np.float32)
    mask = np.zeros((M, o_max), dtype=np.float32)
    y = np.zeros((M, k, scenes.PROP_N_DIM), dtype=np.float32)
    ymask = np.zeros((M, k), dtype=np.float32)
    dmask = np.zeros((M, scenes.PROP_N_DIM), dtype=np.float32)
    ubin = np.zeros(M, dtype=np.int32)
    for i, (p, path) in enumerate(pairs):
        c, o, m = scenes.proposal_features(p, o_max)
        core[i], obs[i], mask[i] = c, o, m
        yy, ym, dm, ub = scenes.proposal_targets(p, path["states"], k)
        y[i], ymask[i], dmask[i], ubin[i] = yy, ym, dm, ub
    return dict(core=core, obs=obs, mask=mask, y=y, ymask=ymask, dmask=dmask, ubin=ubin)


def init_weights(seed=0):
    """He-normal weights, zero biases, the head scaled by 0.1 (flat layout)."""
    rng = np.random.default_rng([0x7EA, seed])
    shapes = [(scenes.PROP_ENC_IN, 64), (96, 256), (256, 256), (256, 256), (256, 256), (256, ST_MLP_OUTPUTS)]
    parts = []
    for li, (fi, fo) in enumerate(shapes):
        w = rng.normal(size=(fi, fo)) * math.sqrt(2.0 / fi)
        if li == len(shapes) - 1:
            w *= 0.1
        parts += [w.astype(np.float32).ravel(), np.zeros(fo, dtype=np.float32)]
    return np.concatenate(parts)


def train(data, steps=3000, batch=256, lr=1e-3, seed=0, weights=None, val_frac=0.1, log=print):
    """Adam on the device.  Returns (weights, history)."""
    import torch
    M = data["core"].shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(M)
    n_val = max(1, int(M * val_frac)) if M > 10 else 0
    val, tr = perm[:n_val], perm[n_val:]
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in data.items()}
    net = Mlp(max(batch, n_val, 1), data["obs"].shape[1])
    net.set_params(weights if weights is not None else init_weights(seed))
    hist = []

    def rows(idx):
        ii = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int64)).cuda()
        return [dev[k].index_select(0, ii).contiguous() for k in ("core", "obs", "mask", "y", "ymask", "dmask",
                                                                  "ubin")]

    def val_loss():
        if n_val == 0:
            return float("nan")
        c, o, m, y, ym, dm, ub = rows(val)
        net.forward(c, o, m)
        return float(net.loss(y, ym, dm, ub).mean())

    t0 = time.time()
    for step in range(steps):
        idx = tr[rng.integers(0, len(tr), size=min(batch, len(tr)))]
        c, o, m, y, ym, dm, ub = rows(idx)
        net.forward(c, o, m)
        per = net.loss(y, ym, dm, ub)
        net.backward()
        # cosine decay to 10 % of the initial rate
        net.adam(lr * (0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * step / max(1, steps)))))
        if step % 250 == 0 or step == steps - 1:
            tl = float(per.mean())
            vl = val_loss()
            hist.append((step, tl, vl))
            log("[train] step %d loss %.4f val %.4f (%.1f s)" % (step, tl, vl, time.time() - t0))
    w = net.get_params()
    net.close()
    return w, hist


class Proposal:
    """Trained weights on the device; installs per-problem outputs."""

    def __init__(self, weights, max_batch=512, o_max=O_MAX):
        self.net = Mlp(max_batch, o_max)
        self.net.set_params(np.asarray(weights, dtype=np.float32))
        self.o_max = o_max

    def outputs(self, problems):
        """Network outputs z [P, 168] (device) for a list of scenes.Problem."""
        import torch
        feats = [scenes.proposal_features(p, self.o_max) for p in problems]
        core = torch.from_numpy(np.stack([f[0] for f in feats]).astype(np.float32)).cuda()
        obs = torch.from_numpy(np.stack([f[1] for f in feats]).astype(np.float32)).cuda()
        mask = torch.from_numpy(np.stack([f[2] for f in feats]).astype(np.float32)).cuda()
        return self.net.forward(core, obs, mask)

    def install(self, gps, problems, mix=0.5):
        """Evaluate the network once per problem and switch its draws on."""
        z = self.outputs(problems)
        for i, gp in enumerate(gps):
            gp.set_proposal(z[i].contiguous(), mix)
        return z


def load_pairs(path, log=print):
    """(problem, path) pairs saved by --save-paths.  A problem is its seed's
    scene (obstacles do not depend on the start/goal draw) with the start and
    goal its path begins and ends at."""
    with np.load(path, allow_pickle=False) as z:
        seeds, lengths, states = z["seeds"], z["lengths"], z["states"]
    out, off = [], 0
    for i, (seed, n) in enumerate(zip(seeds, lengths)):
        st = states[off:off + int(n)]
        off += int(n)
        p = scenes.arm6(int(seed))
        p.q_start = scenes.f32(st[0, :p.d])
        p.q_goal = scenes.f32(st[-1, :p.d])
        p.params.batch = 512
        p.params.cap_fwd = 1 << 16
        p.params.cap_bwd = 1 << 13
        out.append((p, {"states": st}))
        if (i + 1) % 4000 == 0:
            log("[load] %d earlier paths" % (i + 1))
    return out


def load_weights(path):
    return np.load(path, allow_pickle=False).astype(np.float32)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--paths", type=int, default=20000)
    ap.add_argument("--per-batch", type=int, default=128)
    ap.add_argument("--plan-ms", type=float, default=2500.0)
    ap.add_argument("--harvest-s", type=float, default=600.0, help="wall-time cap of the harvest")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--out", required=True)
    ap.add_argument("--log", default=None)
    ap.add_argument("--save-paths", default=None, help="also keep the harvested (seed, path) pairs (.npz)")
    ap.add_argument("--seed0", type=int, default=TRAIN_SEED0, help="first training problem seed")
    ap.add_argument("--with-paths", default=None,
                    help="earlier harvested pairs (.npz from --save-paths) to train on as well")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    earlier = load_pairs(a.with_paths, log=log) if a.with_paths else []
    pairs = harvest(max(a.paths - len(earlier), 0), a.per_batch, a.plan_ms, seed0=a.seed0, log=log,
                    time_limit_s=a.harvest_s)
    if a.save_paths:
        np.savez_compressed(a.save_paths, seeds=np.array([p.seed for p, _ in pairs]),
                            lengths=np.array([len(q["states"]) for _, q in pairs]),
                            states=np.concatenate([q["states"] for _, q in pairs]))
    pairs = earlier + pairs
    data = make_dataset(pairs)
    w, hist = train(data, steps=a.steps, log=log)
    np.save(a.out, w)
    meta = dict(paths=len(pairs), steps=a.steps, history=hist, seconds=time.time() - t0,
                train_seed0=TRAIN_SEED0)
    with open(os.path.splitext(a.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log("[done] %d paths, %d steps, %.0f s" % (len(pairs), a.steps, time.time() - t0))
    return 0


if __name__ == "__main__":
    sys.exit(main())
