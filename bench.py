"""Benchmark of the space-time extend path on one MI355X.

A step is one planner iteration of the whole hot path on the 6-DOF arm
workload (UR5e-like arm as 40 spheres, 16 moving sphere obstacles with 8
waypoints, interval root with 8 groups, 4096 samples per iteration, edge step
0.02 rad): sampling, nearest-node scans, steering, extension edge checks,
insertion, bridge selection and checks, incumbent publish and allocation
update.  `value` is space-time edge checks decided per second over the timed
steps (extension and bridge edges), with the problem resident in HBM.

Printed as one JSON line; see the fields for the roofline of the dominant
kernel, the oracle's throughput on the host cores, the stage breakdown and
the median time to first solution.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published vector FP32 peak
PEAK_HBM_GBS = 8000.0


def flops_per_state(prob) -> int:
    """Algorithmic FP32 flops to decide one space-time state (multiply and add
    count one each; compares and transcendental functions are not counted):
      forward kinematics  69 per joint (3x4 affine product 63 + 6 for A_i),
      sphere centres      18 per sphere (3x3 product and translation),
      obstacle centres     7 per obstacle (segment offset and 3 fused lerps),
      sphere pairs         8 per pair (3 differences, 3 squares, 2 sums)."""
    S, O, d = prob.n_spheres, prob.n_obs, prob.d
    fk = 69 * d if prob.kind == 1 else 3
    sph = 18 * S if prob.kind == 1 else 3 * S
    return fk + sph + 7 * O + 8 * S * O


def pick_problem(maker, lib, first_seed=0, need_solvable=False, limit=64):
    """First seed whose start state is free at t = 0 and whose goal is free at
    some grid time (checked with the library's own kernels)."""
    import torch
    for seed in range(first_seed, first_seed + limit):
        prob = maker(seed)
        gp = lib.Problem(prob)
        x = torch.tensor(np.r_[prob.q_start, 0.0][None], dtype=torch.float32, device="cuda")
        free = gp.check_states(x).cpu().numpy()[0]
        if free and gp.goal_free().any():
            return seed, prob, gp
        gp.close()
    raise RuntimeError("no usable problem found")


def cpu_baseline(prob, seconds=12.0):
    """The FP64 oracle planner on the same problem, single thread, timed on the
    host for a bounded number of whole iterations."""
    import oracle
    op = oracle.Planner(prob)
    t0 = time.perf_counter()
    it = 0
    while time.perf_counter() - t0 < seconds:
        s = op.sample(it)
        op.extend(s)
        it += 1
    dt = time.perf_counter() - t0
    inf = op.info()
    edges = inf["edge_checks"] + inf["bridge_checks"]
    return dict(value=edges / dt, unit="edge checks/s", cores=1, kind="oracle",
                sample="%d planner iterations (B=%d) of the same 6-DOF arm problem from an empty forest, "
                       "FP64 single thread, %.1f s, %d edges" % (it, prob.params.batch, dt, edges))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--roofline-steps", type=int, default=10)
    ap.add_argument("--ttfs-problems", type=int, default=12)
    ap.add_argument("--ttfs-ms", type=float, default=1500.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (problems shard across GPUs "
              "without exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_30533_amd import lib, scenes
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.init()

    seed, prob, gp = pick_problem(scenes.arm6, lib)
    W = flops_per_state(prob)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        # timed region: the production path (captured iteration graphs)
        gp.iterate(args.warmup, stream=stream)
        stream.synchronize()
        w0 = gp.work_counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gp.iterate(args.steps, stream=stream)
        stream.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        w1 = gp.work_counters()
        # event-timed pass over the next iterations of the same plan: HIP events
        # recorded on the launch stream between the pipeline stages give the
        # edge-check launch durations for the roofline
        gp.profile(True)
        p0 = gp.work_counters()
        gp.iterate(args.roofline_steps, stream=stream)
        stream.synchronize()
        stages = gp.profile_read()
        p1 = gp.work_counters()
        gp.profile(False)
    elapsed = t1 - t0
    edges = (w1["edges"] - w0["edges"]) + (w1["bridges"] - w0["bridges"])
    value = edges / elapsed
    states = (p1["edge_states"] - p0["edge_states"]) + (p1["bridge_states"] - p0["bridge_states"])
    ms_edge = stages["edge_check"][0] + stages["bridge_check"][0]
    launches = stages["edge_check"][1] + stages["bridge_check"][1]
    flops = states * W
    achieved = flops / (ms_edge * 1e-3) / 1e12 if ms_edge > 0 else 0.0
    dominant = max(stages, key=lambda k: stages[k][0])
    inf = gp.info()

    # time to first solution, plain sampler, one problem at a time
    ttfs, solved, tried = [], 0, 0
    s = seed
    while tried < args.ttfs_problems:
        try:
            s, p2, g2 = pick_problem(scenes.arm6, lib, first_seed=s + 1)
        except RuntimeError:
            break
        tried += 1
        res = g2.plan(max_ms=args.ttfs_ms, stop_at_first=True, iters_per_sync=1)
        if res["first_iter"] >= 0:
            solved += 1
            ttfs.append(res["first_ms"])
        g2.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, args.cpu_seconds)

    out = {
        "metric": "space-time edge checks/s; median first-solution ms, learned+batched vs plain",
        "value": value,
        "unit": "edge checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "arm6: 6-DOF UR5e-like arm, 40 spheres, 16 moving spheres x 8 waypoints, "
                               "interval root N=8, B=4096, h=0.02 rad, eta=0.5",
                   "problem_seed": seed, "batch": prob.params.batch, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_check_edges (extension + bridge launches)",
                     "flops_per_state": W, "states": states, "launches": launches,
                     "avg_launch_ms": ms_edge / max(launches, 1),
                     "timing": "HIP events on the launch stream around each edge-check launch, %d iterations "
                               "after the timed steps" % args.roofline_steps},
        "cpu_baseline": cpu,
        "stages_ms": {k: round(v[0], 4) for k, v in stages.items()},
        "dominant_stage": dominant,
        "edges_per_step": edges / args.steps,
        "tree_nodes": int(sum(gp.export()["counts"])),
        "ttfs_ms_median_plain": float(np.median(ttfs)) if ttfs else None,
        "ttfs_ms_mean_plain": float(np.mean(ttfs)) if ttfs else None,
        "ttfs_solved": solved,
        "ttfs_problems": tried,
        "incumbent_U": inf["U"] if math.isfinite(inf["U"]) else None,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
