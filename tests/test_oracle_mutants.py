"""The oracle's pins catch the mistakes they claim to catch.

Each case copies the oracle's C source, plants one plausible mistake by a
textual replacement, builds the copy with gcc into a temporary directory,
loads it in place of the real oracle and reruns the pin that names the
mistake: the pin must fail.  The real oracle is restored afterwards.  Only
the CPU is involved.
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from tests import oracle_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "st_oracle.c")
HDR = os.path.join(ROOT, "oracle", "st_oracle.h")

# (id, pin, [(text in the oracle, planted text, expected occurrences)])
MUTANTS = [
    ("bridge-rho-before-arrival", "bridge_ranking",
     [("if (arr < ba || (arr == ba && r < br)) { ba = arr; br = r; best = idx; }",
       "if (r < br || (r == br && arr < ba)) { ba = arr; br = r; best = idx; }", 1)]),
    ("bridge-arrival-from-own-tree", "bridge_ranking",
     [("double arr = sigma > 0 ? p->rootT[idx] : x_rootT;", "double arr = x_rootT;", 2)]),
    ("bridge-keeps-inactive-trees", "bridge_ranking",
     [("if (sigma > 0 && sc->variant == ORC_IR && !(p->rootT[idx] < U)) continue;", "(void)U;", 2)]),
    ("bridge-same-side", "bridge_ranking",
     [("int pool_lo = sigma > 0 ? 1 : 0, pool_hi = sigma > 0 ? p->n_pools : 1;",
       "int pool_lo = sigma > 0 ? 0 : 1, pool_hi = sigma > 0 ? 1 : p->n_pools;", 1)]),
    ("eq8-untruncated-timing", "eq8_max_speed_step",
     [("k->xnew[d] = k->xn[d] + sigma * config_dist(d, k->xn, k->xnew) / v;",
       "k->xnew[d] = k->xn[d] + sigma * Dn / v;", 1)]),
    ("eq8-no-eta-cap", "eq8_max_speed_step",
     [("double f = fmin(1.0, sc->eta / Dn);", "double f = 1.0;", 1)]),
    ("eq8-time-always-forward", "eq8_max_speed_step",
     [("k->xnew[d] = k->xn[d] + sigma * config_dist(d, k->xn, k->xnew) / v;",
       "k->xnew[d] = k->xn[d] + config_dist(d, k->xn, k->xnew) / v;", 1)]),
    ("eq8-parent-by-rho", "eq8_max_speed_step",
     [("NULL, sigma, ORC_METRIC_CONFIG, xr, &Dn, &k->amb);", "NULL, sigma, ORC_METRIC_RHO, xr, &Dn, &k->amb);", 1)]),
    ("validator-no-time-check", "validator_rejections", [("if (!(dtt > 0.0)) FAIL(", "if (0) FAIL(", 1)]),
    ("validator-no-collision-check", "validator_rejections",
     [("if (!orc_edge_check(sc, a, b, &fh, NULL, NULL, NULL)) FAIL",
       "if (0 && !orc_edge_check(sc, a, b, &fh, NULL, NULL, NULL)) FAIL", 1)]),
    ("validator-no-range-check", "validator_rejections",
     [("if (n > 1 && (U < L - 1e-6", "if (0 && n > 1 && (U < L - 1e-6", 1)]),
    ("validator-no-length-check", "validator_rejections",
     [("if (fabs(len - C) > rel_tol", "if (0 && fabs(len - C) > rel_tol", 1)]),
    ("validator-no-start-check", "validator_rejections",
     [("if (fabs(st[j] - sc->q_s[j]) > 1e-6) FAIL", "if (0) FAIL", 1)]),
    ("validator-no-goal-check", "validator_rejections",
     [("if (fabs(last[j] - sc->q_g[j]) > 1e-6) FAIL", "if (0) FAIL", 1)]),
    ("validator-no-start-time-check", "validator_rejections", [("if (fabs(st[d]) > 1e-9) FAIL", "if (0) FAIL", 1)]),
    ("validator-no-arrival-check", "validator_rejections",
     [("if (fabs(last[d] - U) > 1e-6 * fmax(1.0, U)) FAIL", "if (0) FAIL", 1)]),
    ("capacity-claim-not-advanced-on-drop", "capacity_suffix",
     [("claimed[pool] += need;\n            if (claimed[pool] > p->cap[pool]) {",
       "if (p->count[pool] + need > p->cap[pool]) {", 1)]),
    ("capacity-virtual-root-one-slot", "capacity_suffix",
     [("int need = k->parent < 0 ? 2 : 1;", "int need = 1;", 1)]),
    ("learned-log-sd-as-sd", "learned_draw_moments",
     [("p->prop_sd[i] = exp(z[72 + i]);", "p->prop_sd[i] = z[72 + i];", 1)]),
    ("learned-no-pi-scale", "learned_draw_moments",
     [("q[j] = PI * (p->prop_mu[c * 8 + j] + p->prop_sd[c * 8 + j] * nrm[j]);",
       "q[j] = (p->prop_mu[c * 8 + j] + p->prop_sd[c * 8 + j] * nrm[j]);", 1)]),
    ("learned-half-turn-box-muller", "learned_draw_moments",
     [("double th = 2.0 * PI * unit24(u[17 + 2 * k]);", "double th = PI * unit24(u[17 + 2 * k]);", 1)]),
    ("learned-component-off-by-one", "learned_draw_moments",
     [("while (c < 7 && !(unit24(u[14]) < p->prop_wcum[c])) ++c;",
       "while (c < 7 && !(unit24(u[14]) < p->prop_wcum[c + 1])) ++c;", 1)]),
    ("learned-bin-off-by-one", "learned_draw_moments",
     [("while (b < 31 && !(unit24(u[15]) < p->prop_hcum[b])) ++b;",
       "while (b < 31 && !(unit24(u[15]) < p->prop_hcum[b + 1])) ++b;", 1)]),
    ("recycle-init-ignores-free", "recycling_worked_example",
     [("            if (!p->gfree[k - p->k_lo]) continue;\n            xg[p->sc.d] = grid_time(p, k);\n            p->slotT[s] = xg[p->sc.d];\n            p->slotK[s] = k;\n            p->slot_active[s] = 1;\n            push_node(p, 1 + s, xg, -1, 0.0, xg[p->sc.d]);\n            break;\n        }\n    }\n    rr_refresh_active(p);\n}\n\n/* Root recycling",
       "            xg[p->sc.d] = grid_time(p, k);\n            p->slotT[s] = xg[p->sc.d];\n            p->slotK[s] = k;\n            p->slot_active[s] = 1;\n            push_node(p, 1 + s, xg, -1, 0.0, xg[p->sc.d]);\n            break;\n        }\n    }\n    rr_refresh_active(p);\n}\n\n/* Root recycling", 1)]),
    ("recycle-occupied-strata-not-skipped", "recycling_worked_example",
     [("        if (occupied) continue;\n", "        (void)occupied;\n", 1)]),
    ("recycle-strata-below-H", "recycling_worked_example",
     [("while (k_end <= p->k_hi && grid_time(p, k_end) < U) ++k_end;",
       "while (k_end <= p->k_hi && grid_time(p, k_end) < p->H) ++k_end;", 1)]),
    ("recycle-generation-kept", "recycling_worked_example",
     [("            p->slot_gen[s]++;\n", "", 1)]),
    ("recycle-donors-in-reverse", "recycling_worked_example",
     [("            int s = donors[di++];", "            int s = donors[nd - 1 - di++];", 1)]),
    ("learned-wrong-mix", "learned_draw_moments",
     [("const int use_net = learned && unit24(u[13]) < p->prop_mix;",
       "const int use_net = learned && unit24(u[13]) < 0.5;", 1)]),
]


def _build_mutant(tmp, edits):
    src = open(SRC).read()
    for old, new, count in edits:
        assert src.count(old) == count, "mutation anchor not found as expected: %r" % old
        src = src.replace(old, new)
    os.makedirs(tmp, exist_ok=True)
    with open(os.path.join(tmp, "st_oracle.c"), "w") as f:
        f.write(src)
    shutil.copy(HDR, os.path.join(tmp, "st_oracle.h"))
    so = os.path.join(tmp, "libmutant.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-w", "-o", so,
                           os.path.join(tmp, "st_oracle.c"), "-lm"])
    return so


@pytest.mark.parametrize("mid,pin,edits", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pin_catches_mutant(oracle_lib, tmp_path, mid, pin, edits):
    from oracle import binding
    so = _build_mutant(str(tmp_path), edits)
    lib = C.CDLL(so)
    binding._declare(lib)
    saved = binding._lib
    binding._lib = lib
    try:
        with pytest.raises(AssertionError):
            oracle_pins.PINS[pin](oracle_lib)
    finally:
        binding._lib = saved


def test_unmutated_copy_passes(oracle_lib, tmp_path):
    """The harness itself: a copy built the same way without a planted
    mistake passes every pin."""
    from oracle import binding
    so = _build_mutant(str(tmp_path), [])
    lib = C.CDLL(so)
    binding._declare(lib)
    saved = binding._lib
    binding._lib = lib
    try:
        for pin in oracle_pins.PINS.values():
            pin(oracle_lib)
    finally:
        binding._lib = saved
