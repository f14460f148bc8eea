"""Autotuner of the many-problem launch: samples per problem per iteration
and lanes per bridge chunk, chosen per problem class and cached as JSON.

A class is (degrees of freedom, obstacle-count bucket).  For each class the
tuner draws tuning problems of that class (seeds disjoint from evaluation
seeds), plans them as one batch under each candidate setting for a fixed
device-time budget, and scores a setting by the summed time to first
solution (an unsolved problem counts the whole budget).  It searches the
sample count first with 16 lanes per bridge chunk, then the lane count at
the best sample count.  (Extension edges take the flattened path, where the
lanes per chunk play no part.)  Everything it runs is the library's planner;
this module only orders the experiments and keeps the table.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import scenes
from .lib import Batch, Problem

SAMPLES = (64, 128, 256, 512)
LANES = (8, 16, 32, 64)
LANES_FIRST = 16
OBS_BUCKETS = (8, 16, 32, 64)
TUNE_SEED0 = 3_000_000
DEFAULT = {"samples": 128, "lanes_extension": 32, "lanes_bridge": 16}


def obs_bucket(n_obs: int) -> int:
    for b in OBS_BUCKETS:
        if n_obs <= b:
            return b
    return OBS_BUCKETS[-1]


def class_key(prob: scenes.Problem) -> str:
    return "d%d-o%d" % (prob.d, obs_bucket(prob.n_obs))


def tuning_problems(key: str, n: int, seed0: int = TUNE_SEED0, max_draws: int = 200000):
    """n problems of the mixed workload that fall in class `key`."""
    out = []
    s = seed0
    while len(out) < n and s < seed0 + max_draws:
        p = scenes.mixed(s)
        s += 1
        if class_key(p) == key:
            out.append(p)
    return out


def apply(prob: scenes.Problem, table: dict, gp: Problem | None = None):
    """Set the problem's sample count (before creation) and, given its
    handle, its launch shape, from the table entry of its class."""
    e = table.get(class_key(prob), DEFAULT)
    prob.params.batch = int(e["samples"])
    if gp is not None:
        gp.set_tuning(lanes_extension=int(e["lanes_extension"]), lanes_bridge=int(e["lanes_bridge"]))
    return e


def score(problems, samples, lanes, budget_ms):
    for p in problems:
        p.params.batch = samples
    gps = [Problem(p, problem_id=i) for i, p in enumerate(problems)]
    for g in gps:
        g.set_tuning(lanes_extension=DEFAULT["lanes_extension"], lanes_bridge=lanes)
    b = Batch(gps)
    r = b.plan(max_ms=budget_ms, stop_at_first=True)
    fm = np.where(np.isfinite(r["first_ms"]), r["first_ms"], budget_ms)
    b.close()
    for g in gps:
        g.close()
    return float(np.minimum(fm, budget_ms).sum()), int(r["n_solved"])


def tune(keys, n_problems=48, budget_ms=400.0, log=print):
    table = {}
    for key in keys:
        probs = tuning_problems(key, n_problems)
        if not probs:
            continue
        best = None
        for smp in SAMPLES:
            sc, ns = score(probs, smp, LANES_FIRST, budget_ms)
            log("[tune] %s samples %d bridge lanes %d: score %.1f solved %d" % (key, smp, LANES_FIRST, sc, ns))
            if best is None or sc < best[0]:
                best = (sc, smp, LANES_FIRST)
        for ln in LANES:
            if ln == LANES_FIRST:
                continue
            sc, ns = score(probs, best[1], ln, budget_ms)
            log("[tune] %s samples %d bridge lanes %d: score %.1f solved %d" % (key, best[1], ln, sc, ns))
            if sc < best[0]:
                best = (sc, best[1], ln)
        table[key] = {"samples": best[1], "lanes_extension": DEFAULT["lanes_extension"], "lanes_bridge": best[2],
                      "score": best[0]}
    return table


def all_keys():
    return ["d%d-o%d" % (d, o) for d in (2, 6, 7) for o in OBS_BUCKETS]


def load(path):
    with open(path) as f:
        return json.load(f)


def main(argv=None):
    ap = argparse.ArgumentParser(description="tune samples per problem and lanes per edge for batched launches")
    ap.add_argument("--out", required=True)
    ap.add_argument("--problems", type=int, default=48)
    ap.add_argument("--budget-ms", type=float, default=400.0)
    ap.add_argument("--keys", default=None, help="comma-separated classes (default: all)")
    a = ap.parse_args(argv)
    keys = a.keys.split(",") if a.keys else all_keys()
    t0 = time.time()
    table = tune(keys, a.problems, a.budget_ms, log=lambda m: print(m, flush=True))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("[tune] %d classes in %.0f s -> %s" % (len(table), time.time() - t0, a.out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
