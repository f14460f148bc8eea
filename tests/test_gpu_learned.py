"""The trained proposal network: the paths it is trained on are valid for the
oracle, and on evaluation problems (seeds disjoint from the training range)
mixing it 50/50 with the plain sampler finds first solutions sooner without
solving fewer problems, every path again valid for the oracle."""
import math
import os

import numpy as np
import pytest

from paper_2609_30533_amd import proposal, scenes
from tests.gpu_util import banner, torch_cuda

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(proposal.__file__), "data", "proposal_arm6.npy")


def test_harvested_paths_are_oracle_valid(oracle_lib):
    torch_cuda()
    banner("harvest")
    pairs = proposal.harvest(12, per_batch=128, max_ms=300.0, log=lambda m: None, time_limit_s=60)
    assert len(pairs) >= 6
    for p, path in pairs:
        assert p.params.seed is not None and path["states"].shape[1] == p.d + 1
        ok, msg = oracle_lib.Oracle(p).validate_path(path["states"], path["U"], path["C"], rel_tol=1e-4)
        assert ok, msg
    data = proposal.make_dataset(pairs)
    assert np.all(data["ymask"].sum(axis=1) >= 2)
    assert np.all((data["ubin"] >= 0) & (data["ubin"] < scenes.PROP_N_BINS))


def _eval(lib, seeds, prop, budget_ms):
    probs = []
    for s in seeds:
        p = scenes.arm6(s)
        p.params.batch = 256
        p.params.cap_fwd = 1 << 16
        p.params.cap_bwd = 1 << 13
        probs.append(p)
    gps = [lib.Problem(p, problem_id=i) for i, p in enumerate(probs)]
    if prop is not None:
        prop.install(gps, probs, 0.5)
    b = lib.Batch(gps)
    r = b.plan(max_ms=budget_ms)
    return probs, gps, b, r


def test_learned_proposal_gains(oracle_lib):
    from paper_2609_30533_amd import lib
    torch_cuda()
    assert os.path.exists(WEIGHTS), "trained weights missing"
    prop = proposal.Proposal(proposal.load_weights(WEIGHTS), max_batch=256)
    seeds = list(range(256))
    banner("learned vs plain on %d evaluation problems" % len(seeds))
    _, gpa, ba, ra = _eval(lib, seeds, None, 1500.0)
    probs, gpl, bl, rl = _eval(lib, seeds, prop, 1500.0)
    fa, fl = ra["first_ms"], rl["first_ms"]
    common = np.isfinite(fa) & np.isfinite(fl)
    banner("plain solved %d median %.1f ms; learned solved %d median %.1f ms; common %d" % (
        ra["n_solved"], np.median(fa[np.isfinite(fa)]), rl["n_solved"], np.median(fl[np.isfinite(fl)]), common.sum()))
    assert common.sum() >= 10
    assert rl["n_solved"] >= ra["n_solved"] - 2
    assert np.median(fl[common]) < np.median(fa[common])
    for i in np.where(np.isfinite(fl))[0]:
        path = gpl[i].path()
        ok, msg = oracle_lib.Oracle(probs[i]).validate_path(path["states"], path["U"], path["C"], rel_tol=1e-4)
        assert ok, (i, msg)
    ba.close()
    bl.close()
