"""Benchmark of the space-time extend path on one MI355X.

A step is one planner iteration of the whole hot path on the 6-DOF arm
workload (UR5e-like arm as 40 spheres, 16 moving sphere obstacles with 8
waypoints, interval root with 8 groups, 4096 samples per iteration, edge step
0.02 rad): sampling, nearest-node scans, steering, extension edge checks,
insertion, bridge selection and checks, incumbent publish and allocation
update.  `value` is space-time edge checks decided per second over the timed
steps (extension and bridge edges), with the problem resident in HBM.

Printed as one JSON line; see the fields for the roofline of the dominant
kernel, the oracle's throughput on the host cores, the stage breakdown, the
median time to first solution of the plain planner (one problem at a time)
against the learned proposal in a batch of many problems, and the
heterogeneous batch's edge-check throughput.
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
# HBM bytes per edge-check launch (average of an extension and a bridge launch)
# from the FETCH_SIZE / WRITE_SIZE profiles of the current kernels, scaled by a
# plain copy kernel of known size (profiles/traffic_arm6_single.md); to be
# measured again whenever the edge-check kernels change.
EDGE_LAUNCH_HBM_BYTES = 1.681e6


def flops_per_state(prob) -> int:
    """Algorithmic FP32 flops to decide one space-time state (multiply and add
    count one each; compares and transcendental functions are not counted):
      forward kinematics  69 per joint (3x4 affine product 63 + 6 for A_i),
      sphere centres      18 per sphere (3x3 product and translation),
      obstacle centres     7 per obstacle (segment offset and 3 fused lerps),
      sphere pairs         8 per pair (3 differences, 3 squares, 2 sums).
    With static geometry (arms) also
      link pairs          63 per listed pair (relative frame), 18 per sphere of
                          the upper link, 8 per sphere pair,
      boxes               26 per sphere and box (axis offsets 18, excess and
                          squared distance 8)."""
    S, O, d = prob.n_spheres, prob.n_obs, prob.d
    fk = 69 * d if prob.kind == 1 else 3
    sph = 18 * S if prob.kind == 1 else 3 * S
    w = fk + sph + 7 * O + 8 * S * O
    links = np.asarray(prob.sphere_link)
    for la, lb in {tuple(p) for p in np.asarray(getattr(prob, "self_pairs", np.zeros((0, 2)))).tolist()}:
        na, nb = int((links == la).sum()), int((links == lb).sum())
        if na and nb:
            w += 63 + 18 * nb + 8 * na * nb
    w += 26 * S * len(getattr(prob, "boxes", ()))
    return int(w)


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


def eval_problem(seed, B=256, cap_fwd=1 << 16, cap_bwd=1 << 13):
    """An evaluation problem of the 6-DOF arm workload (seeds below the
    training and tuning ranges) with the batch's sample count and capacities."""
    from paper_2609_30533_amd import scenes
    p = scenes.arm6(seed)
    p.params.batch = B
    p.params.cap_fwd = cap_fwd
    p.params.cap_bwd = cap_bwd
    return p


def batched_run(lib, probs, budget_ms, proposal=None, mix=0.5, table=None):
    """Plan all problems as one batch; returns the batch result and the summed
    work counters of its members."""
    from paper_2609_30533_amd import autotune
    if table is not None:
        for p in probs:
            autotune.apply(p, table)
    gps = [lib.Problem(p, problem_id=i) for i, p in enumerate(probs)]
    if table is not None:
        for p, g in zip(probs, gps):
            autotune.apply(p, table, g)
    if proposal is not None:
        proposal.install(gps, probs, mix)
    b = lib.Batch(gps)
    w0 = [g.work_counters() for g in gps]
    r = b.plan(max_ms=budget_ms)
    w1 = [g.work_counters() for g in gps]
    edges = sum((a["edges"] - z["edges"]) + (a["bridges"] - z["bridges"]) for a, z in zip(w1, w0))
    states = sum((a["edge_states"] - z["edge_states"]) + (a["bridge_states"] - z["bridge_states"])
                 for a, z in zip(w1, w0))
    b.close()
    for g in gps:
        g.close()
    r["edges"] = edges
    r["states"] = states
    return r


def ttfs_section(lib, args):
    """Median time to first solution: plain sampler one problem at a time
    (the paper's setting) against the learned proposal in a batch of many
    problems, on the same evaluation seeds."""
    from paper_2609_30533_amd import proposal
    P = args.ttfs_batch
    wpath = os.path.join(ROOT, "paper_2609_30533_amd", "data", "proposal_arm6.npy")
    prop = proposal.Proposal(proposal.load_weights(wpath), max_batch=P)
    seeds = list(range(P))
    plain_b = batched_run(lib, [eval_problem(s) for s in seeds], args.ttfs_ms)
    learned_b = batched_run(lib, [eval_problem(s) for s in seeds], args.ttfs_ms, proposal=prop)
    fp, fl = plain_b["first_ms"], learned_b["first_ms"]
    solvable = [s for i, s in enumerate(seeds) if math.isfinite(fp[i]) or math.isfinite(fl[i])]
    single = {}
    for mode in ("plain", "learned"):
        t, U = {}, {}
        for s in solvable:
            p = eval_problem(s, B=4096, cap_fwd=1 << 18, cap_bwd=1 << 16)
            g = lib.Problem(p)
            if mode == "learned":
                prop.install([g], [p], 0.5)
            r = g.plan(max_ms=args.ttfs_single_ms, stop_at_first=True, iters_per_sync=1)
            if r["first_iter"] >= 0:
                t[s], U[s] = r["first_ms"], r["U"]
            g.close()
        single[mode] = (t, U)
    tp, Up = single["plain"]
    common = [s for s in solvable if s in tp and math.isfinite(fl[s])]

    # the same comparison as a workload: the first Q evaluation problems
    # submitted together; plain answers them one after another (each with its
    # budget), the learned batch answers them all at once.  A problem's time
    # is from the submission of the workload to its first solution.
    Q = args.queue_problems
    queue = {}
    if Q > 0:
        t0 = time.perf_counter()
        for s in range(Q):
            p = eval_problem(s, B=4096, cap_fwd=1 << 18, cap_bwd=1 << 16)
            g = lib.Problem(p)
            ts = (time.perf_counter() - t0) * 1e3
            r = g.plan(max_ms=args.queue_ms, stop_at_first=True, iters_per_sync=1)
            if r["first_iter"] >= 0:
                queue[s] = ts + r["first_ms"]
            g.close()
        plain_queue_wall = (time.perf_counter() - t0) * 1e3
        lq = batched_run(lib, [eval_problem(s) for s in range(Q)], args.queue_ms, proposal=prop)
        qcommon = [s for s in queue if math.isfinite(lq["first_ms"][s])]

    def med(v):
        return float(np.median(v)) if len(v) else None

    return {
        "ttfs_workload": "arm6 evaluation seeds 0..%d (6-DOF arm, 16 moving spheres); plain = one problem at a "
                         "time, B=4096, %.0f ms budget; batched = all %d problems in one batch, B=256 each, "
                         "%.0f ms budget; learned = proposal network mixed 50/50" % (
                             P - 1, args.ttfs_single_ms, P, args.ttfs_ms),
        "ttfs_solvable": len(solvable),
        "ttfs_common": len(common),
        "ttfs_ms_median_plain": med([tp[s] for s in common]),
        "ttfs_ms_median_learned_batched": med([fl[s] for s in common]),
        "ttfs_ms_median_plain_batched": med([fp[s] for s in common if math.isfinite(fp[s])]),
        "ttfs_ms_median_learned_single": med([single["learned"][0][s] for s in common if s in single["learned"][0]]),
        "arrival_mean_plain": med([]) if not common else float(np.mean([Up[s] for s in common])),
        "arrival_mean_learned_batched": float(np.mean([learned_b["U"][s] for s in common])) if common else None,
        "solved_plain_single": len(tp),
        "solved_learned_single": len(single["learned"][0]),
        "solved_plain_batched": int(plain_b["n_solved"]),
        "solved_learned_batched": int(learned_b["n_solved"]),
        "batched_wall_ms": float(learned_b["total_ms"]),
        "plain_sequential_wall_ms_solvable": float(sum(tp.values()) + args.ttfs_single_ms * (len(solvable) - len(tp))),
        "queue_workload": "the first %d evaluation problems submitted at once; %.0f ms budget per problem (plain, "
                          "one after another) or for the whole batch (learned+batched); time from submission to "
                          "each problem's first solution, median over problems both solve" % (Q, args.queue_ms),
        "queue_ms_median_plain": med([queue[s] for s in qcommon]) if Q > 0 else None,
        "queue_ms_median_learned_batched": med([float(lq["first_ms"][s]) for s in qcommon]) if Q > 0 else None,
        "queue_common": len(qcommon) if Q > 0 else 0,
        "queue_wall_ms_plain": plain_queue_wall if Q > 0 else None,
        "queue_wall_ms_learned_batched": float(lq["total_ms"]) if Q > 0 else None,
    }


def batched_section(lib, args):
    """The heterogeneous batch: 512 problems (DOF 2/6/7, 4-64 obstacles,
    arrival widths 5-60 s, capacities 2^14-2^18) in one batch, samples per
    problem and lanes per edge from the tuning table."""
    from paper_2609_30533_amd import autotune, scenes
    tpath = os.path.join(ROOT, "paper_2609_30533_amd", "data", "tuning.json")
    table = autotune.load(tpath) if os.path.exists(tpath) else {}
    probs = [scenes.mixed(s) for s in range(args.batch_problems)]
    r = batched_run(lib, probs, args.batch_ms, table=table)
    fm = r["first_ms"][np.isfinite(r["first_ms"])]
    return {
        "batched_workload": "mixed seeds 0..%d: DOF 2/6/7, 4-64 obstacles, arrival widths 5-60 s, tree "
                            "capacity 2^14-2^18, one batch, %.0f ms" % (args.batch_problems - 1, args.batch_ms),
        "batched_edge_checks_per_s": r["edges"] / (r["total_ms"] * 1e-3),
        "batched_iterations": int(r["iterations"]),
        "batched_solved": int(r["n_solved"]),
        "batched_ttfs_ms_median": float(np.median(fm)) if len(fm) else None,
        "batched_states": int(r["states"]),
        "tuning_table": "paper_2609_30533_amd/data/tuning.json" if table else None,
    }


def edge_sweep(lib, scenes, n_edges, reps=5):
    """st_check_edges on n_edges synthetic speed-feasible edges of the 6-DOF
    arm problem (lengths up to 4 eta) for each obstacle tile and lane count:
    the edge-check kernel with the whole device to itself.  Algorithmic work
    is the states up to the first hit (all n+1 for a free edge)."""
    import torch
    prob = scenes.arm6(1)
    xa, xb = scenes.synthetic_edges(prob, n_edges, seed=5, bridge_mix=True)
    # state counts n = max(1, ceil(max(D, v dt) / h)) of the edges, host side
    D = np.sqrt(((xb[:, :-1].astype(np.float64) - xa[:, :-1]) ** 2).sum(axis=1))
    span = np.maximum(D, prob.v_max * np.abs(xb[:, -1].astype(np.float64) - xa[:, -1]))
    n = np.maximum(1, np.ceil(span / prob.params.h)).astype(np.int64)
    da, db = torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda()
    gp = lib.Problem(prob)
    W = flops_per_state(prob)
    out = []
    for ot in (8, 16):
        for lanes in (16, 32, 64):
            gp.set_tuning(obstacle_tile=ot, lanes_check=lanes)
            free, fh = gp.check_edges(da, db)
            torch.cuda.synchronize()
            fh = fh.cpu().numpy()
            states = int(np.where(fh < 0, n + 1, fh + 1).sum())
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(reps):
                gp.check_edges(da, db)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / reps
            tf = states * W / (ms * 1e-3) / 1e12
            out.append(dict(obstacle_tile=ot, lanes=lanes, ms=ms, states=states, edges=n_edges,
                            tflops=tf, frac=tf / PEAK_FP32_TFLOPS))
    gp.close()
    return out


def ablation(lib, scenes, args):
    """Allocation ablation (Sec. VI): root recycling against fixed roots
    (deactivation only) as the arrival range widens, 16 roots and 512
    samples per iteration, on disc problems whose obstacles move during the
    first 10 s (the 7-DOF stand-ins are rarely solvable); each condition is
    one batch of the same problems with the same budget; mean final arrival
    over the problems both solve."""
    out = []
    for H in (10.0, 25.0, 50.0, 100.0):
        res = {}
        for nr in (0, 1):
            probs = []
            for s in range(args.ablation):
                p = scenes.disc2d(s, horizon=10.0, t_min=0.0,
                                  params=scenes.Params(variant=scenes.VARIANT_RR, n_groups=16, batch=512, eta=0.1,
                                                       h=0.01, cap_fwd=1 << 16, cap_bwd=1 << 12, seed=1,
                                                       no_recycling=nr))
                p.t_max = scenes.f32(H)
                probs.append(p)
            res[nr] = batched_run(lib, probs, args.ablation_ms)
        both = np.isfinite(res[0]["U"]) & np.isfinite(res[1]["U"])
        out.append({"workload": "disc2d, 8 moving discs, range [0, %g] s" % H, "roots": 16, "samples": 512,
                    "budget_ms": args.ablation_ms, "problems": args.ablation,
                    "solved_recycling": int(res[0]["n_solved"]), "solved_no_recycling": int(res[1]["n_solved"]),
                    "common": int(both.sum()),
                    "mean_arrival_recycling": float(np.mean(res[0]["U"][both])) if both.any() else None,
                    "mean_arrival_no_recycling": float(np.mean(res[1]["U"][both])) if both.any() else None})
    return out


def single_run(gp, prob, args):
    """The timed steps of one problem (captured iteration graphs on a side
    stream) and an event-timed pass over the following iterations."""
    import torch
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
    states = (p1["edge_states"] - p0["edge_states"]) + (p1["bridge_states"] - p0["bridge_states"])
    ms_edge = stages["edge_check"][0] + stages["bridge_check"][0]
    launches = stages["edge_check"][1] + stages["bridge_check"][1]
    achieved = states * W / (ms_edge * 1e-3) / 1e12 if ms_edge > 0 else 0.0
    return dict(elapsed=elapsed, edges=edges, value=edges / elapsed, states=states, ms_edge=ms_edge,
                launches=launches, stages=stages, flops_per_state=W, achieved=achieved)


def report(args, seed, prob, gp, m, ttfs, batched, cpu):
    elapsed, edges, value, states, ms_edge, launches, stages = (m[k] for k in (
        "elapsed", "edges", "value", "states", "ms_edge", "launches", "stages"))
    W, achieved = m["flops_per_state"], m["achieved"]
    dominant = max(stages, key=lambda k: stages[k][0])
    inf = gp.info()
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
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": EDGE_LAUNCH_HBM_BYTES,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE, copy-scaled)",
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
        "incumbent_U": inf["U"] if math.isfinite(inf["U"]) else None,
    }
    out.update(ttfs)
    out.update(batched)
    print(json.dumps(out))


def static_section(lib, scenes, args):
    """Self-collision and fixed boxes (the 6-DOF arm with its listed link
    pairs, a table and a post): the single-problem step throughput on the
    same configuration as the headline, and time to first solution of a batch
    of problems with and without the static terms."""
    seed, prob, gp = pick_problem(scenes.arm6static, lib)
    m = single_run(gp, prob, args)
    gp.close()
    print(json.dumps({"workload": "arm6 with self-collision (10 link pairs) and 2 fixed boxes, interval root N=8, "
                                  "B=4096", "problem_seed": seed, "edge_checks_per_s": m["value"],
                      "ms_per_step": m["elapsed"] * 1e3 / args.steps, "flops_per_state": m["flops_per_state"],
                      "edge_check_tflops": m["achieved"], "frac": m["achieved"] / PEAK_FP32_TFLOPS,
                      "stages_ms": {k: round(v[0], 4) for k, v in m["stages"].items()}}), flush=True)
    # evaluation problems whose start and goal clear the static terms (and the
    # moving obstacles at t = 0), checked with the library's kernels
    import torch
    seeds = []
    s = 0
    while len(seeds) < args.static and s < 50 * args.static:
        p = scenes.with_static(eval_problem(s))
        g = lib.Problem(p)
        x = torch.tensor(np.r_[p.q_start, 0.0][None], dtype=torch.float32, device="cuda")
        if g.check_states(x).cpu().numpy()[0] and g.goal_free().any():
            seeds.append(s)
        g.close()
        s += 1
    res = {}
    for st in (0, 1):
        probs = [scenes.with_static(eval_problem(s)) if st else eval_problem(s) for s in seeds]
        res[st] = batched_run(lib, probs, args.static_ms)
    fm = [r["first_ms"] for r in (res[0], res[1])]
    both = np.isfinite(fm[0]) & np.isfinite(fm[1])
    print(json.dumps({"workload": "%d arm6 problems (B=256) as one batch, %g ms budget, start and goal clear of "
                                  "the static terms" % (len(seeds), args.static_ms),
                      "solved_plain": int(res[0]["n_solved"]), "solved_static": int(res[1]["n_solved"]),
                      "median_first_ms_plain": float(np.median(fm[0][both])) if both.any() else None,
                      "median_first_ms_static": float(np.median(fm[1][both])) if both.any() else None,
                      "common": int(both.sum()),
                      "edges_per_s_plain": res[0]["edges"] / max(res[0]["total_ms"], 1e-9) * 1e3,
                      "edges_per_s_static": res[1]["edges"] / max(res[1]["total_ms"], 1e-9) * 1e3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--roofline-steps", type=int, default=10)
    ap.add_argument("--ttfs-batch", type=int, default=512, help="evaluation problems (0: skip the comparison)")
    ap.add_argument("--ttfs-ms", type=float, default=2000.0, help="budget of each batched evaluation run")
    ap.add_argument("--ttfs-single-ms", type=float, default=1000.0, help="budget of each single-problem run")
    ap.add_argument("--queue-problems", type=int, default=128, help="problems of the workload comparison (0: skip)")
    ap.add_argument("--queue-ms", type=float, default=100.0)
    ap.add_argument("--batch-problems", type=int, default=512, help="heterogeneous batch size (0: skip)")
    ap.add_argument("--batch-ms", type=float, default=2000.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-reference", type=int, default=0,
                    help="only copy this many MiB device to device three times (the reference kernel that "
                         "scales the memory counters of a profile) and exit")
    ap.add_argument("--ablation", type=int, default=0,
                    help="only run the recycling ablation on this many problems per condition and print JSON")
    ap.add_argument("--ablation-ms", type=float, default=1000.0)
    ap.add_argument("--edge-sweep", type=int, default=0,
                    help="only time st_check_edges on this many synthetic edges per launch shape and print JSON")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--static", type=int, default=0,
                    help="self-collision and boxes: throughput and a batch of this many problems (0: skip)")
    ap.add_argument("--static-ms", type=float, default=1000.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (problems shard across GPUs "
              "without exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_30533_amd import lib, scenes
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.init()

    if args.copy_reference > 0:
        n = args.copy_reference * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_reference_bytes": n * 4, "copies": 3}))
        return

    if args.ablation > 0:
        for r in ablation(lib, scenes, args):
            print(json.dumps(r), flush=True)
        return

    if args.edge_sweep > 0:
        for r in edge_sweep(lib, scenes, args.edge_sweep):
            print(json.dumps(r), flush=True)
        return

    if args.static > 0:
        static_section(lib, scenes, args)
        return

    seed, prob, gp = pick_problem(scenes.arm6, lib)
    m = single_run(gp, prob, args)
    ttfs = ttfs_section(lib, args) if args.ttfs_batch > 0 else {}
    batched = batched_section(lib, args) if args.batch_problems > 0 else {}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, args.cpu_seconds)
    report(args, seed, prob, gp, m, ttfs, batched, cpu)


if __name__ == "__main__":
    main()
