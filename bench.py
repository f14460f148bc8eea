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
PEAK_BF16_TFLOPS = 2500.0     # MI355X published dense BF16 matrix-core peak
PEAK_HBM_GBS = 8000.0
# Sources of the edge-check kernels: a traffic figure measured with rocprofv3
# counters is reported only while these are unchanged since the measurement.
EDGE_KERNEL_SOURCES = ("paper_2609_30533_amd/csrc/collide.hip", "paper_2609_30533_amd/csrc/edge_flat.hpp",
                       "paper_2609_30533_amd/csrc/extend.hip", "paper_2609_30533_amd/csrc/st_device.hpp")
TRAFFIC_PROFILE = "profiles/traffic_arm6_single.md"


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in EDGE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """(bytes per edge-check launch, provenance) from the committed counter
    profile, or (None, reason) when the kernels changed since it was taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    vals = {}
    try:
        for line in open(path):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    except OSError:
        return None, "no traffic profile"
    if vals.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None, "edge-check kernels changed since %s was measured" % TRAFFIC_PROFILE
    try:
        return float(vals["edge_launch_hbm_bytes"]), TRAFFIC_PROFILE
    except (KeyError, ValueError):
        return None, "no traffic figure in %s" % TRAFFIC_PROFILE


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


def pick_problem(workload, lib, first_seed=0, limit=64, **kw):
    """The first seed whose redrawn start is free at t = 0 and whose goal is
    free at some grid time (both checked with the library's own kernels)."""
    from paper_2609_30533_amd import problems
    for seed in range(first_seed, first_seed + limit):
        prob, _ = problems.eval_problem(workload, seed, **kw)
        if prob is not None:
            return seed, prob, lib.Problem(prob)
    raise RuntimeError("no usable problem found")


def progress(msg):
    """A progress line on stderr (the JSON result stays alone on stdout)."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_planner_rate(prob, seconds):
    """Edges the FP64 oracle planner decides per second on one thread, over
    whole iterations of the problem from an empty forest."""
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
    return edges, dt, it


def _oracle_worker(args):
    prob, seconds = args
    return _oracle_planner_rate(prob, seconds)


def cpu_baseline(prob, seconds=12.0, all_cores=True):
    """The FP64 oracle planner on the same problem, timed on the host for a
    bounded number of whole iterations: one thread, then (all_cores) one
    independent oracle planner per host core at once (aggregate rate)."""
    edges, dt, it = _oracle_planner_rate(prob, seconds)
    out = dict(value=edges / dt, unit="edge checks/s", cores=1, kind="oracle", cpu_model=_cpu_model(),
               sample="%d planner iterations (B=%d) of the same 6-DOF arm problem from an empty forest, "
                      "FP64 single thread, %.1f s, %d edges" % (it, prob.params.batch, dt, edges))
    if all_cores:
        import multiprocessing as mp
        n = min(os.cpu_count() or 1, 16)
        with mp.get_context("spawn").Pool(n) as pool:
            t0 = time.perf_counter()
            res = pool.map(_oracle_worker, [(prob, seconds / 2)] * n)
            wall = time.perf_counter() - t0
        tot = sum(r[0] for r in res)
        out["all_cores"] = dict(value=tot / max(r[1] for r in res), cores=n,
                                sample="%d independent oracle planners on the same problem at once, %.1f s each "
                                       "(%.1f s wall incl. start-up), %d edges" % (n, seconds / 2, wall, tot))
    return out


def eval_problem(seed, B=256, cap_fwd=1 << 16, cap_bwd=1 << 13, planner_seed=1):
    """Evaluation problem `seed` of the 6-DOF arm workload (seeds below the
    training and tuning ranges): start and goal redrawn until the library
    finds the start free at t = 0 and some goal-grid time free; the batch's
    sample count and capacities; the planner's own seed.  None if no draw is
    accepted."""
    from paper_2609_30533_amd import problems
    p, _ = problems.eval_problem("arm6", seed, max_attempts=16)
    if p is None:
        return None
    p.params.batch = B
    p.params.cap_fwd = cap_fwd
    p.params.cap_bwd = cap_bwd
    p.params.seed = planner_seed
    return p


def _with(prob, B, cap_fwd, cap_bwd, planner_seed):
    import copy
    p = copy.deepcopy(prob)
    p.params.batch, p.params.cap_fwd, p.params.cap_bwd, p.params.seed = B, cap_fwd, cap_bwd, planner_seed
    return p


def batched_run(lib, probs, budget_ms, proposal=None, mix=0.5, table=None, keep_paths=False, iters_per_launch=4,
                lanes_bridge=0):
    """Plan all problems as one batch; returns the batch result and the summed
    work counters of its members (keep_paths: the solved members' paths).
    A member's first-solution time is resolved to the launch (graph of
    iters_per_launch iterations) that found it."""
    from paper_2609_30533_amd import autotune
    t_setup = time.perf_counter()
    if table is not None:
        for p in probs:
            autotune.apply(p, table)
    gps = [lib.Problem(p, problem_id=i) for i, p in enumerate(probs)]
    if lanes_bridge:
        for g in gps:
            g.set_tuning(lanes_bridge=lanes_bridge)
    if table is not None:
        for p, g in zip(probs, gps):
            autotune.apply(p, table, g)
    if proposal is not None:
        proposal.install(gps, probs, mix)
    b = lib.Batch(gps, iters_per_launch=iters_per_launch)
    w0 = [g.work_counters() for g in gps]
    # host set-up of the batch (problems, start checks, proposal, graphs)
    setup_ms = (time.perf_counter() - t_setup) * 1e3
    r = b.plan(max_ms=budget_ms)
    r["setup_ms"] = setup_ms
    w1 = [g.work_counters() for g in gps]
    edges = sum((a["edges"] - z["edges"]) + (a["bridges"] - z["bridges"]) for a, z in zip(w1, w0))
    per = [(a["edge_states"] - z["edge_states"]) + (a["bridge_states"] - z["bridge_states"]) for a, z in zip(w1, w0)]
    states = sum(per)
    # algorithmic flops of the decided states, each member at its own cost per state
    flops = sum(n * flops_per_state(p) for n, p in zip(per, probs))
    if keep_paths:
        r["paths"] = {i: g.path() for i, g in enumerate(gps) if r["first_iter"][i] >= 0}
    b.close()
    for g in gps:
        g.close()
    r["edges"] = edges
    r["states"] = states
    r["flops"] = flops
    return r


def _bootstrap_median_diff(a, b, reps=2000, seed=0):
    """Paired bootstrap (resampling (problem, planner seed) pairs) 95 %
    interval of median(b) - median(a) and of median(b) / median(a)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if len(a) < 2:
        return None
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(a), size=(reps, len(a)))
    ma, mb = np.median(a[idx], axis=1), np.median(b[idx], axis=1)
    d, r = mb - ma, mb / np.maximum(ma, 1e-12)
    return {"diff_ms": [float(np.percentile(d, 2.5)), float(np.percentile(d, 97.5))],
            "ratio": [float(np.percentile(r, 2.5)), float(np.percentile(r, 97.5))]}


def _wilcoxon_p(a, b):
    try:
        from scipy.stats import wilcoxon
        if len(a) < 5 or np.allclose(np.asarray(a), np.asarray(b)):
            return None
        return float(wilcoxon(np.asarray(b) - np.asarray(a)).pvalue)
    except Exception:
        return None


def ttfs_section(lib, args, validate):
    """Time to first solution on the evaluation problems (the protocol of the
    paper's evaluation: planner seeds 1-3, common-success sets, bootstrap
    intervals): the plain planner one problem at a time (B = 4096, the
    headline configuration) against the learned proposal with all problems
    in one batch (--ttfs-batch-samples each, mixed 50/50), with two batched controls on
    the same batch: the plain sampler and an untrained network of the same
    architecture.  Both sides are timed on the device from the first
    iteration's launch to the end of the iteration that found a problem's
    first solution (a batch member: from the batch's first launch); the
    set-up before it (start checks, graph capture, proposal) is not counted
    on either side.  Solved paths go to `validate` (the oracle re-checks them
    in the CPU leg)."""
    from paper_2609_30533_amd import proposal
    wpath = os.path.join(ROOT, "paper_2609_30533_amd", "data", "proposal_arm6.npy")
    base = []
    for s in range(args.ttfs_problems):
        p = eval_problem(s)
        if p is not None:
            base.append((s, p))
    n = len(base)
    trained = proposal.Proposal(proposal.load_weights(wpath), max_batch=max(n, 1))
    untrained = proposal.Proposal(proposal.init_weights(seed=77), max_batch=max(n, 1))
    conds = (("plain_batched", None), ("learned_batched", trained), ("untrained_batched", untrained))
    t = {c: {} for c in [c for c, _ in conds] + ["plain"]}     # (problem, planner seed) -> first ms
    U = {c: {} for c in t}                                     # arrival at the end of the run
    it1 = {c: {} for c in t}                                   # iterations to the first solution
    for ps in args.planner_seeds:
        batch_probs = [_with(p, args.ttfs_batch_samples, 1 << 16, 1 << 13, ps) for _, p in base]
        for c, prop in conds:
            progress("time to first solution: planner seed %d, %s batch of %d problems" % (ps, c, n))
            # one iteration per launch: first solutions timed to the iteration
            r = batched_run(lib, batch_probs, args.ttfs_ms, proposal=prop, keep_paths=True, iters_per_launch=1,
                            lanes_bridge=args.ttfs_lanes_bridge)
            for i, path in r["paths"].items():
                key = (base[i][0], ps)
                t[c][key] = float(r["first_ms"][i])
                U[c][key] = float(r["U"][i])
                it1[c][key] = int(r["first_iter"][i])
                if path["rc"] == 0:
                    validate.append((batch_probs[i], path["states"], path["U"], path["C"]))
        solved_any = sorted({k[0] for c, _ in conds for k in t[c] if k[1] == ps})
        progress("time to first solution: planner seed %d, plain one at a time on %d problems" % (ps, len(solved_any)))
        for s in solved_any:
            p = _with(dict(base)[s], 4096, 1 << 18, 1 << 16, ps)
            g = lib.Problem(p)
            if args.ttfs_lanes_bridge:
                g.set_tuning(lanes_bridge=args.ttfs_lanes_bridge)
            r = g.plan(max_ms=args.ttfs_single_ms, stop_at_first=True, iters_per_sync=1)
            if r["first_iter"] >= 0 and r["rc"] == 0:
                t["plain"][(s, ps)] = r["first_ms"]
                U["plain"][(s, ps)] = r["U"]
                it1["plain"][(s, ps)] = int(r["first_iter"])
                validate.append((p, r["states"], r["U"], r["C"]))
            g.close()

    def med(v):
        return float(np.median(v)) if len(v) else None

    def mean(v):
        return float(np.mean(v)) if len(v) else None

    out = {
        "ttfs_workload": "arm6 evaluation seeds 0..%d with start and goal accepted by the library (%d problems), "
                         "planner seeds %s; plain = one problem at a time, B=4096, %.0f ms budget, stop at the "
                         "first solution; batched = all problems in one batch, B=%d each, %.0f ms; learned and "
                         "untrained networks mixed 50/50; %s lanes per bridge chunk in both; a time is device "
                         "time from the first iteration's launch to the end of the iteration that found the "
                         "first solution, the set-up (start check, graph capture, proposal) excluded on both "
                         "sides" % (
                             args.ttfs_problems - 1, n, list(args.planner_seeds), args.ttfs_single_ms,
                             args.ttfs_batch_samples, args.ttfs_ms, args.ttfs_lanes_bridge or "default"),
        "ttfs_problems": n,
        "ttfs_runs": n * len(args.planner_seeds),
    }
    for c in t:
        out["solved_%s" % c] = len(t[c])
    # the headline comparison: learned+batched against plain on their common successes
    common = sorted(set(t["plain"]) & set(t["learned_batched"]))
    a = [t["plain"][k] for k in common]
    b = [t["learned_batched"][k] for k in common]
    out.update({
        "ttfs_common": len(common),
        "ttfs_ms_median_plain": med(a), "ttfs_ms_median_learned_batched": med(b),
        "ttfs_ms_mean_plain": mean(a), "ttfs_ms_mean_learned_batched": mean(b),
        "ttfs_bootstrap95_learned_batched_minus_plain": _bootstrap_median_diff(a, b),
        "ttfs_wilcoxon_p": _wilcoxon_p(a, b),
        # direction of the paired comparison (the Wilcoxon test is two-sided)
        "ttfs_pairs_learned_batched_faster": float(np.mean(np.asarray(b) < np.asarray(a))) if common else None,
        "ttfs_median_paired_diff_ms": float(np.median(np.asarray(b) - np.asarray(a))) if common else None,
    })
    # controls on their own common sets with plain
    for c in ("plain_batched", "untrained_batched"):
        cm = sorted(set(t["plain"]) & set(t[c]))
        out["ttfs_common_%s" % c] = len(cm)
        out["ttfs_ms_median_%s" % c] = med([t[c][k] for k in cm])
        out["ttfs_ms_median_plain_vs_%s" % c] = med([t["plain"][k] for k in cm])
    # learned against untrained and plain sampling in the same batch: time and
    # arrival at the end of the batch's budget, on the problems all three solve
    cb = sorted(set(t["plain_batched"]) & set(t["learned_batched"]) & set(t["untrained_batched"]))
    out["batched_common"] = len(cb)
    for c in ("plain_batched", "learned_batched", "untrained_batched"):
        out["batched_ttfs_ms_median_%s" % c] = med([t[c][k] for k in cb])
        out["batched_first_iter_median_%s" % c] = med([it1[c][k] for k in cb])
        out["batched_first_iter_mean_%s" % c] = mean([it1[c][k] for k in cb])
        out["batched_arrival_mean_%s" % c] = mean([U[c][k] for k in cb])
    out["ttfs_first_iter_median_plain"] = med([it1["plain"][k] for k in common])
    out["batched_bootstrap95_learned_minus_untrained"] = _bootstrap_median_diff(
        [t["untrained_batched"][k] for k in cb], [t["learned_batched"][k] for k in cb])

    # the same comparison as a workload: the first Q evaluation problems
    # submitted together; plain answers them one after another (each with its
    # budget), the learned batch answers them all at once.  A problem's time
    # is from the submission of the workload to its first solution.
    Q = min(args.queue_problems, n)
    if Q > 0:
        queue = {}
        t0 = time.perf_counter()
        for i in range(Q):
            p = _with(base[i][1], 4096, 1 << 18, 1 << 16, 1)
            g = lib.Problem(p)
            r = g.plan(max_ms=args.queue_ms, stop_at_first=True, iters_per_sync=1)
            if r["first_iter"] >= 0:
                # host time at the return of the first solution (with its path)
                queue[i] = (time.perf_counter() - t0) * 1e3
            g.close()
        plain_queue_wall = (time.perf_counter() - t0) * 1e3
        # the batch's set-up (problems, start checks, proposal, graphs) counts
        # too: a member's time is the set-up plus the device time to its first
        # solution
        lq = batched_run(lib, [_with(base[i][1], args.ttfs_batch_samples, 1 << 16, 1 << 13, 1) for i in range(Q)],
                         args.queue_ms, proposal=trained, iters_per_launch=1)
        lq_first = lq["setup_ms"] + lq["first_ms"]
        qcommon = [i for i in queue if math.isfinite(lq_first[i])]
        out.update({
            "queue_workload": "the first %d evaluation problems submitted at once; %.0f ms budget per problem "
                              "(plain, one after another) or for the whole batch (learned+batched); time from "
                              "submission to each problem's first solution, every set-up included (plain: host "
                              "time at the return of its first solution; batched: the batch's host set-up plus "
                              "the device time to the member's first solution), median over problems both "
                              "solve" % (Q, args.queue_ms),
            "queue_ms_median_plain": med([queue[i] for i in qcommon]),
            "queue_ms_median_learned_batched": med([float(lq_first[i]) for i in qcommon]),
            "queue_common": len(qcommon),
            "queue_wall_ms_plain": plain_queue_wall,
            "queue_setup_ms_learned_batched": float(lq["setup_ms"]),
            "queue_wall_ms_learned_batched": float(lq["setup_ms"] + lq["total_ms"]),
        })

    # final arrival at equal time for the workload: the first A evaluation
    # problems, plain one after another with an equal share of the budget each
    # (its start check and graph capture inside its share) against the learned
    # batch with the whole budget (its set-up before it)
    A = min(args.arrival_problems, n)
    if A > 0:
        share = args.arrival_ms / A
        progress("arrival at equal time: %d problems, plain %.1f ms each, learned batch %.0f ms" % (
            A, share, args.arrival_ms))
        up = {}
        for i in range(A):
            p = _with(base[i][1], 4096, 1 << 18, 1 << 16, 1)
            g = lib.Problem(p)
            r = g.plan(max_ms=share, iters_per_sync=8)
            if r["rc"] == 0 and r["first_iter"] >= 0:
                up[i] = float(r["U"])
                validate.append((p, r["states"], r["U"], r["C"]))
            g.close()
        bp = [_with(base[i][1], args.ttfs_batch_samples, 1 << 16, 1 << 13, 1) for i in range(A)]
        lb = batched_run(lib, bp, args.arrival_ms, proposal=trained, keep_paths=True,
                         lanes_bridge=args.ttfs_lanes_bridge)
        ub = {}
        for i, path in lb["paths"].items():
            if path["rc"] == 0:
                ub[i] = float(path["U"])
                validate.append((bp[i], path["states"], path["U"], path["C"]))
        ac = sorted(set(up) & set(ub))
        out.update({
            "arrival_workload": "the first %d evaluation problems, %.0f ms in all: plain one after another with "
                                "%.1f ms each (set-up inside), learned+batched with the whole budget; mean final "
                                "arrival over problems both solve" % (A, args.arrival_ms, share),
            "arrival_solved_plain": len(up), "arrival_solved_learned_batched": len(ub), "arrival_common": len(ac),
            "arrival_mean_plain": mean([up[i] for i in ac]),
            "arrival_mean_learned_batched": mean([ub[i] for i in ac]),
            "arrival_pairs_learned_batched_earlier": float(np.mean([ub[i] < up[i] for i in ac])) if ac else None,
        })
    return out


def batched_section(lib, args):
    """The heterogeneous batch: 512 problems (DOF 2/6/7, 4-64 obstacles,
    arrival widths 5-60 s, capacities 2^14-2^18) in one batch, samples per
    problem and lanes per edge from the tuning table."""
    from paper_2609_30533_amd import autotune, scenes
    tpath = os.path.join(ROOT, "paper_2609_30533_amd", "data", "tuning.json")
    table = autotune.load(tpath) if os.path.exists(tpath) else {}
    probs = [scenes.mixed(s) for s in range(args.batch_problems)]
    for p in probs:
        # one obstacle tile for the whole batch: the members' kernel instances
        # then differ only by robot kind (two scene classes instead of six)
        p.params.obstacle_tile = args.batch_obstacle_tile
    r = batched_run(lib, probs, args.batch_ms, table=table)
    fm = r["first_ms"][np.isfinite(r["first_ms"])]
    return {
        "batched_workload": "mixed seeds 0..%d: DOF 2/6/7, 4-64 obstacles, arrival widths 5-60 s, tree "
                            "capacity 2^14-2^18, one batch, %.0f ms, obstacle tile %s" % (
                                args.batch_problems - 1, args.batch_ms, args.batch_obstacle_tile or "per problem"),
        "batched_edge_checks_per_s": r["edges"] / (r["total_ms"] * 1e-3),
        "batched_iterations": int(r["iterations"]),
        "batched_solved": int(r["n_solved"]),
        "batched_ttfs_ms_median": float(np.median(fm)) if len(fm) else None,
        "batched_states": int(r["states"]),
        # the members' states differ in cost (2-DOF discs to 7-DOF arms against
        # 64 obstacles): the algorithmic rate over the whole batched run
        "batched_edge_check_tflops": r["flops"] / (r["total_ms"] * 1e-3) / 1e12,
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


def gemm_flops(M, O):
    """Matrix-core flops of one training step of the proposal network (2 m n k
    per product): forward through the encoder (M*O obstacle rows, 65 -> 64),
    the four hidden layers (96 -> 256, then 256 -> 256) and the head
    (256 -> 168); backward the weight gradient of every layer and the input
    gradient of every layer but the encoder."""
    enc, din, w, out = (65, 64), 96, 256, 168
    f = 2 * M * O * enc[0] * enc[1] + 2 * M * din * w + 3 * 2 * M * w * w + 2 * M * w * out
    b = 2 * w * out * M + 2 * M * out * w                       # head: dW5, dh4
    b += 3 * (2 * w * w * M + 2 * M * w * w)                      # layers 4..2: dW, dX
    b += 2 * din * w * M + 2 * M * w * din                        # layer 1: dW, dx0
    b += 2 * enc[0] * enc[1] * M * O                              # encoder dW
    return f, b


def gemm_bench(lib, rows_list, steps, O=32):
    """Training steps of the proposal network (forward, loss, backward, Adam)
    on random rows, timed with HIP events on the launch stream; the
    algorithmic matrix-core work against MI355X's dense BF16 peak."""
    import torch
    out = []
    for M in rows_list:
        net = lib.Mlp(M, O)
        rng = np.random.default_rng(3)
        from paper_2609_30533_amd import proposal
        net.set_params(proposal.init_weights(seed=5))
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
        core, obs = dev(rng.normal(size=(M, 16)) * 0.3), dev(rng.normal(size=(M, O, 65)) * 0.3)
        mask = dev(np.ones((M, O)))
        y, ym = dev(rng.normal(size=(M, 16, 8)) * 0.3), dev(np.ones((M, 16)))
        dm = dev(np.ones((M, 8)))
        ub = torch.from_numpy(rng.integers(0, 32, size=M).astype(np.int32)).cuda()
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            for _ in range(3):
                net.forward(core, obs, mask, stream=stream)
                net.loss(y, ym, dm, ub, stream=stream)
                net.backward(stream=stream)
                net.adam(1e-4, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                net.forward(core, obs, mask, stream=stream)
                net.loss(y, ym, dm, ub, stream=stream)
                net.backward(stream=stream)
                net.adam(1e-4, stream=stream)
            e1.record(stream)
            stream.synchronize()
        ms = e0.elapsed_time(e1) / steps
        f, b = gemm_flops(M, O)
        tf = (f + b) / (ms * 1e-3) / 1e12
        out.append({"rows": M, "obstacles": O, "ms_per_step": ms, "gemm_gflop_per_step": (f + b) / 1e9,
                    "tflops": tf, "peak_bf16_tflops": PEAK_BF16_TFLOPS, "frac": tf / PEAK_BF16_TFLOPS})
        net.close()
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


def config_rows(lib, args):
    """The single-problem step on the two other configurations, each with
    its own edge-check roofline: the disc workload (2 DOF, 8 discs at
    constant velocity, B = 256) and the recycling workload at its own shape
    (7 DOF, 60 spheres, 32 obstacles x 16 waypoints, 64 slots, B = 8192)."""
    rows = []
    for wl, label in (("disc2d", "disc2d: disc robot in the unit square, 8 discs at constant velocity, interval root "
                                 "N=4, B=256, h=0.01"),
                      ("arm7rr", "arm7rr: 7-DOF arm, 60 spheres, 32 moving spheres x 16 waypoints, root recycling "
                                 "with 64 slots, B=8192, h=0.02 rad")):
        # the first accepted problem whose planner still works during the
        # timed steps (an interval-root plan whose incumbent reaches the lower
        # bound L stops: L >= min(H, U))
        first = 0
        for _ in range(8):
            seed, prob, gp = pick_problem(wl, lib, first_seed=first)
            m = single_run(gp, prob, args)
            gp.close()
            if m["edges"] > 0:
                break
            first = seed + 1
        rows.append({"workload": label, "problem_seed": seed, "edge_checks_per_s": m["value"],
                     "ms_per_step": m["elapsed"] * 1e3 / args.steps, "flops_per_state": m["flops_per_state"],
                     "roofline": {"bound": "alu", "achieved": m["achieved"], "peak": PEAK_FP32_TFLOPS,
                                  "unit": "TFLOP/s", "frac": m["achieved"] / PEAK_FP32_TFLOPS,
                                  "states": m["states"], "launches": m["launches"],
                                  "avg_launch_ms": m["ms_edge"] / max(m["launches"], 1)},
                     "edges_per_step": m["edges"] / args.steps})
    return rows


def report(args, seed, prob, gp, m, ttfs, batched, cpu, configs):
    elapsed, edges, value, states, ms_edge, launches, stages = (m[k] for k in (
        "elapsed", "edges", "value", "states", "ms_edge", "launches", "stages"))
    W, achieved = m["flops_per_state"], m["achieved"]
    dominant = max(stages, key=lambda k: stages[k][0])
    inf = gp.info()
    traffic, traffic_src = measured_traffic()
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
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, copy-scaled)",
                     "traffic_source": traffic_src,
                     "kernel": "edge check: extension launch k_steer_flat (steering fused with the check), "
                               "bridge launch k_bridge_check (merge fused with the first 64 states) + k_edge_items",
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
    out["configs"] = configs
    out.update(ttfs)
    out.update(batched)
    print(json.dumps(out))


def static_section(lib, scenes, args):
    """Self-collision and fixed boxes (the 6-DOF arm with its listed link
    pairs, a table and a post): the single-problem step throughput on the
    same configuration as the headline, and time to first solution of a batch
    of problems with and without the static terms."""
    seed, prob, gp = pick_problem("arm6static", lib)
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
        p0 = eval_problem(s)
        if p0 is None:
            s += 1
            continue
        p = scenes.with_static(p0)
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
    ap.add_argument("--ttfs-problems", type=int, default=300, help="evaluation problems (0: skip the comparison)")
    ap.add_argument("--planner-seeds", type=lambda v: [int(x) for x in v.split(",")], default=[1, 2, 3])
    ap.add_argument("--ttfs-ms", type=float, default=1000.0, help="budget of each batched evaluation run")
    ap.add_argument("--ttfs-single-ms", type=float, default=1000.0, help="budget of each single-problem run")
    ap.add_argument("--no-configs", action="store_true", help="skip the disc and recycling configuration rows")
    ap.add_argument("--queue-problems", type=int, default=128, help="problems of the workload comparison (0: skip)")
    ap.add_argument("--queue-ms", type=float, default=100.0)
    ap.add_argument("--arrival-problems", type=int, default=128,
                    help="problems of the equal-time arrival comparison (0: skip)")
    ap.add_argument("--arrival-ms", type=float, default=2560.0, help="budget of the whole arrival workload")
    ap.add_argument("--batch-problems", type=int, default=512, help="heterogeneous batch size (0: skip)")
    ap.add_argument("--batch-ms", type=float, default=2000.0)
    ap.add_argument("--batch-obstacle-tile", type=int, default=16,
                    help="obstacle tile forced on every member of the heterogeneous batch (0: each its own)")
    ap.add_argument("--ttfs-lanes-bridge", type=int, default=32,
                    help="lanes per bridge chunk of every time-to-first-solution problem, plain and batched "
                         "(0: the library's default)")
    ap.add_argument("--ttfs-batch-samples", type=int, default=32,
                    help="samples per iteration of each problem in the time-to-first-solution batches")
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
    ap.add_argument("--gemm-steps", type=int, default=0,
                    help="only time this many proposal-network training steps (256 and 16384 rows) and print JSON")
    ap.add_argument("--static", type=int, default=0,
                    help="self-collision and boxes: throughput and a batch of this many problems (0: skip)")
    ap.add_argument("--static-ms", type=float, default=1000.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (independent problems would "
              "shard across GPUs without exchange)", file=sys.stderr)
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

    if args.gemm_steps > 0:
        for r in gemm_bench(lib, (256, 16384), args.gemm_steps):
            print(json.dumps(r), flush=True)
        return

    if args.edge_sweep > 0:
        for r in edge_sweep(lib, scenes, args.edge_sweep):
            print(json.dumps(r), flush=True)
        return

    if args.static > 0:
        static_section(lib, scenes, args)
        return

    # the headline problem: the first seed of the arm workload whose own draw
    # of start and goal is accepted (seed 1)
    seed, prob, gp = pick_problem("arm6", lib, first_seed=1)
    progress("headline: %d warm-up and %d timed iterations" % (args.warmup, args.steps))
    m = single_run(gp, prob, args)
    progress("headline: %.4f ms per iteration" % (m["elapsed"] * 1e3 / args.steps))
    configs = [] if args.no_configs else config_rows(lib, args)
    to_validate = []
    ttfs = ttfs_section(lib, args, to_validate) if args.ttfs_problems > 0 else {}
    if args.batch_problems > 0:
        progress("heterogeneous batch of %d problems" % args.batch_problems)
    batched = batched_section(lib, args) if args.batch_problems > 0 else {}
    cpu = None
    if not args.no_cpu_baseline:
        progress("oracle baseline on the host cores")
        cpu = cpu_baseline(prob, args.cpu_seconds)
        progress("oracle re-validation of %d paths" % len(to_validate))
        # every compared path re-checked by the oracle
        import oracle
        bad = [i for i, (p, st, U, C) in enumerate(to_validate)
               if not oracle.Oracle(p).validate_path(st, U, C, rel_tol=1e-4)[0]]
        ttfs["paths_validated"] = len(to_validate)
        ttfs["paths_invalid"] = len(bad)
    report(args, seed, prob, gp, m, ttfs, batched, cpu, configs)


if __name__ == "__main__":
    main()
