"""st_check_edges_noalloc (the edge check with a fixed work area, for callers
that cannot allocate) against st_check_edges on the same inputs: identical
free flags and first hits, on two calls in a row with the second smaller,
and against the oracle on edges whose clearance is not fragile."""
import numpy as np
import pytest

from paper_2609_30533_amd import scenes
from tests.gpu_util import banner, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("make", [lambda: scenes.arm6(3), lambda: scenes.disc2d(2)], ids=["arm6", "disc2d"])
def test_noalloc_matches_check_edges(oracle_lib, make):
    from paper_2609_30533_amd import lib
    torch = torch_cuda()
    prob = make()
    prob.params.cap_fwd, prob.params.cap_bwd = 1 << 12, 1 << 10
    gp = lib.Problem(prob)
    o = oracle_lib.Oracle(prob)
    E_max = lib.NOALLOC_MAX_EDGES
    free = torch.full((E_max,), 7, dtype=torch.uint8, device="cuda")
    fh = torch.full((E_max,), -7, dtype=torch.int32, device="cuda")
    for call, (E, seed) in enumerate([(E_max, 31), (3001, 32)]):
        banner("noalloc %s call %d: %d edges" % (prob.name, call, E))
        xa, xb = scenes.synthetic_edges(prob, E, seed=seed, bridge_mix=True)
        da, db = to_dev(xa), to_dev(xb)
        ref_free, ref_fh = gp.check_edges(da, db)
        gp.check_edges_noalloc(da, db, free[:E], fh[:E])
        torch.cuda.synchronize()
        assert torch.equal(free[:E], ref_free) and torch.equal(fh[:E], ref_fh)
        # and against the oracle on a sample of edges away from contact
        idx = np.random.default_rng(seed).choice(E, size=min(E, 400), replace=False)
        r = o.check_edges(xa[idx].astype(np.float64), xb[idx].astype(np.float64))
        sure = r["margin"] > 1e-4
        f = free[:E].cpu().numpy()[idx]
        h = fh[:E].cpu().numpy()[idx]
        assert np.array_equal(f[sure], r["free"][sure])
        assert np.array_equal(h[sure], r["first_hit"][sure])
        assert sure.sum() > 0.5 * len(idx)
    # beyond the fixed work area: an error, nothing launched
    xa, xb = scenes.synthetic_edges(prob, E_max + 1, seed=33)
    with pytest.raises(lib.StError, match="fixed work area"):
        gp.check_edges_noalloc(to_dev(xa), to_dev(xb), torch.empty(E_max + 1, dtype=torch.uint8, device="cuda"))
