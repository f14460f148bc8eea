"""Evaluation problem sets: seeded problems whose start and goal the library's
own kernels accept.

The paper assumes every query has a free start and a goal that is free at
some time in the arrival range.  Random start/goal pairs among moving
spheres often violate that, which makes most of a seeded set unsolvable for
every planner alike.  These helpers redraw a problem's start and goal (its
obstacles unchanged) until the start is free at t = 0 and some goal-grid time
k dt in the search domain is free, both decided by the HIP kernels of the
library (the state check and the goal grid computed when a problem is
created).  No planning arithmetic lives here.
"""
from __future__ import annotations

import copy

import numpy as np

from . import lib, scenes


def start_goal_ok(prob: scenes.Problem) -> bool:
    """True when the library finds the start free at t = 0 and at least one
    free goal-grid time (a throwaway handle with small pools)."""
    import torch
    probe = copy.deepcopy(prob)
    probe.params.cap_fwd = 256
    probe.params.cap_bwd = 64
    gp = lib.Problem(probe)
    try:
        if not gp.goal_free().any():
            return False
        x = torch.tensor(np.r_[prob.q_start, 0.0][None, :], dtype=torch.float32, device="cuda")
        return bool(gp.check_states(x).cpu().numpy()[0])
    finally:
        gp.close()


def eval_problem(workload: str, seed: int, max_attempts: int = 64, **kw):
    """Problem `seed` of a workload with its start and goal redrawn until the
    library accepts them; (problem, attempt) or (None, max_attempts)."""
    make = scenes.WORKLOADS[workload]
    return scenes.redraw_until(lambda a: make(seed, attempt=a, **kw), start_goal_ok, max_attempts)
