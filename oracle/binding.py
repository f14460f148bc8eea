"""ctypes binding of the FP64 C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "st_oracle.c")
_BUILD = os.path.join(_HERE, "_build")

MAX_DOF, MAX_SPH, MAX_OBS, MAX_WP = 7, 128, 64, 32
MAX_SELF, MAX_BOX = 32, 16


def lib_path() -> str:
    return os.path.join(_BUILD, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2, scalar FP64)."""
    out = lib_path()
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    os.makedirs(_BUILD, exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-fno-fast-math",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)
    return out


class Scene(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("kind", C.c_int32),
        ("dh", C.c_double * 4 * MAX_DOF),
        ("n_sph", C.c_int32),
        ("sph_link", C.c_int32 * MAX_SPH),
        ("sph", C.c_double * 4 * MAX_SPH),
        ("q_lo", C.c_double * MAX_DOF), ("q_hi", C.c_double * MAX_DOF),
        ("q_s", C.c_double * MAX_DOF), ("q_g", C.c_double * MAX_DOF),
        ("t_min", C.c_double), ("t_max", C.c_double), ("v_max", C.c_double),
        ("n_obs", C.c_int32),
        ("n_wp", C.c_int32 * MAX_OBS),
        ("wp", C.c_double * 4 * MAX_WP * MAX_OBS),
        ("obs_r", C.c_double * MAX_OBS),
        ("variant", C.c_int32), ("n_groups", C.c_int32), ("batch", C.c_int32),
        ("eta", C.c_double), ("h", C.c_double), ("dt", C.c_double),
        ("p_new", C.c_double), ("p_guided", C.c_double),
        ("cap_fwd", C.c_int32), ("cap_bwd", C.c_int32),
        ("seed", C.c_uint32), ("problem_id", C.c_uint32), ("no_recycling", C.c_int32),
        ("n_self", C.c_int32), ("self_pair", C.c_int32 * 2 * MAX_SELF),
        ("n_box", C.c_int32), ("box", C.c_double * 15 * MAX_BOX),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = lib_path()
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


P = np.ctypeslib.ndpointer
f64 = P(dtype=np.float64, flags="C_CONTIGUOUS")
i32 = P(dtype=np.int32, flags="C_CONTIGUOUS")
i64 = P(dtype=np.int64, flags="C_CONTIGUOUS")
u8 = P(dtype=np.uint8, flags="C_CONTIGUOUS")
i8 = P(dtype=np.int8, flags="C_CONTIGUOUS")
u32 = P(dtype=np.uint32, flags="C_CONTIGUOUS")


def _opt(t):
    """ndpointer that also accepts None."""
    class _O(t):  # type: ignore[misc, valid-type]
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return t.from_param(obj)
    return _O


def _declare(L):
    S = C.POINTER(Scene)
    L.orc_philox4x32_10.argtypes = [u32, u32, u32]
    L.orc_frames.argtypes = [S, f64, f64]
    L.orc_sphere_centres.argtypes = [S, f64, f64]
    L.orc_obstacle_pos.argtypes = [S, C.c_int, C.c_double, f64]
    L.orc_state_valid.argtypes = [S, f64, C.POINTER(C.c_double)]
    L.orc_state_valid.restype = C.c_int
    L.orc_check_edges.argtypes = [S, C.c_int64, f64, f64, u8, _opt(i32), _opt(i64), _opt(f64), _opt(f64)]
    L.orc_check_states.argtypes = [S, C.c_int64, f64, u8, _opt(f64)]
    L.orc_edge_continuous.argtypes = [S, f64, f64, C.POINTER(C.c_double)]
    L.orc_edge_continuous.restype = C.c_int
    L.orc_edge_continuous_pw.argtypes = [S, f64, f64, C.POINTER(C.c_double)]
    L.orc_edge_continuous_pw.restype = C.c_int
    L.orc_rho.argtypes = [C.c_int, C.c_double, C.c_int, f64, f64]
    L.orc_rho.restype = C.c_double
    L.orc_nearest.argtypes = [S, C.c_int64, f64, _opt(u8), C.c_int, C.c_int, f64, C.POINTER(C.c_double),
                              C.POINTER(C.c_uint8)]
    L.orc_nearest.restype = C.c_int64
    L.orc_lower_bound.argtypes = [S]
    L.orc_lower_bound.restype = C.c_double
    L.orc_goal_grid_range.argtypes = [S, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.orc_goal_grid.argtypes = [S, C.c_int64, C.c_int64, u8]
    L.orc_ir_partition.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64, u8,
                                   C.c_int, f64, i32, f64, C.c_int]
    L.orc_ir_partition.restype = C.c_int
    L.orc_planner_create.argtypes = [S]
    L.orc_planner_create.restype = C.c_void_p
    L.orc_planner_destroy.argtypes = [C.c_void_p]
    L.orc_planner_sample.argtypes = [C.c_void_p, C.c_int64, C.c_int64, i8, u8, i32, f64, f64, f64]
    L.orc_planner_extend.argtypes = [C.c_void_p, C.c_int64, i8, u8, i32, f64, f64, f64,
                                     _opt(i8), _opt(i32), _opt(i32), _opt(f64), _opt(i32), _opt(u8), _opt(f64),
                                     _opt(f64), _opt(u8), _opt(f64), _opt(f64)]
    L.orc_planner_extend.restype = C.c_int
    L.orc_planner_run.argtypes = [C.c_void_p, C.c_int64]
    L.orc_planner_run.restype = C.c_int
    L.orc_planner_path.argtypes = [C.c_void_p, C.c_int64, f64]
    L.orc_planner_path.restype = C.c_int64
    L.orc_planner_info.argtypes = [C.c_void_p, f64]
    L.orc_planner_counts.argtypes = [C.c_void_p, i64]
    L.orc_planner_goal_free.argtypes = [C.c_void_p, u8]
    L.orc_planner_partition.argtypes = [C.c_void_p, f64, i32, f64, C.c_int]
    L.orc_planner_slots.argtypes = [C.c_void_p, f64, i32, u32, i64]
    L.orc_planner_export.argtypes = [C.c_void_p, f64, i32, f64, f64]
    L.orc_planner_import.argtypes = [C.c_void_p, i64, f64, i32, f64, f64, C.c_double, C.c_double, C.c_int64,
                                     C.c_int64, C.c_int64, _opt(f64), _opt(i32), _opt(u32), _opt(i64)]
    L.orc_planner_bridge.argtypes = [C.c_void_p, C.c_int, f64, C.c_double, C.POINTER(C.c_double),
                                     C.POINTER(C.c_uint8)]
    L.orc_planner_bridge.restype = C.c_int64
    L.orc_planner_recycle.argtypes = [C.c_void_p, C.c_double]
    L.orc_planner_recycle.restype = C.c_int
    L.orc_planner_set_proposal.argtypes = [C.c_void_p, _opt(f64), C.c_double]
    L.orc_validate_path.argtypes = [S, C.c_int64, f64, C.c_double, C.c_double, C.c_double, C.c_char_p, C.c_int]
    L.orc_validate_path.restype = C.c_int


def make_scene(prob, problem_id: int = 0) -> Scene:
    """Fill the oracle's scene record from a generated problem."""
    s = Scene()
    s.d, s.kind = prob.d, prob.kind
    for i in range(prob.d):
        for j in range(4):
            s.dh[i][j] = float(prob.dh[i, j])
    s.n_sph = prob.n_spheres
    for k in range(prob.n_spheres):
        s.sph_link[k] = int(prob.sphere_link[k])
        for j in range(4):
            s.sph[k][j] = float(prob.sphere[k, j])
    for j in range(prob.d):
        s.q_lo[j], s.q_hi[j] = float(prob.q_lo[j]), float(prob.q_hi[j])
        s.q_s[j], s.q_g[j] = float(prob.q_start[j]), float(prob.q_goal[j])
    s.t_min, s.t_max, s.v_max = float(prob.t_min), float(prob.t_max), float(prob.v_max)
    s.n_obs = prob.n_obs
    for o in range(prob.n_obs):
        s.n_wp[o] = int(prob.n_wp[o])
        s.obs_r[o] = float(prob.obs_r[o])
        for k in range(int(prob.n_wp[o])):
            for j in range(4):
                s.wp[o][k][j] = float(prob.wp[o, k, j])
    p = prob.params
    s.variant, s.n_groups, s.batch = p.variant, p.n_groups, p.batch
    s.eta, s.h, s.dt, s.p_new, s.p_guided = p.eta, p.h, p.dt, p.p_new, p.p_guided
    s.cap_fwd, s.cap_bwd = p.cap_fwd, p.cap_bwd
    s.seed, s.problem_id = p.seed & 0xFFFFFFFF, problem_id & 0xFFFFFFFF
    s.no_recycling = 1 if getattr(p, "no_recycling", 0) else 0
    pairs = np.asarray(getattr(prob, "self_pairs", np.zeros((0, 2))), dtype=np.int64).reshape(-1, 2)
    boxes = np.asarray(getattr(prob, "boxes", np.zeros((0, 15))), dtype=np.float64).reshape(-1, 15)
    assert len(pairs) <= MAX_SELF and len(boxes) <= MAX_BOX
    s.n_self = len(pairs)
    for k, (a, b) in enumerate(pairs):
        s.self_pair[k][0], s.self_pair[k][1] = int(a), int(b)
    s.n_box = len(boxes)
    for k in range(len(boxes)):
        for j in range(15):
            s.box[k][j] = float(boxes[k, j])
    return s


class Oracle:
    """Stateless geometry / check / metric functions for one scene."""

    def __init__(self, prob, problem_id: int = 0):
        self.lib = _load()
        self.prob = prob
        self.scene = make_scene(prob, problem_id)
        self.d = prob.d

    # geometry --------------------------------------------------------------
    def frames(self, q):
        out = np.zeros((self.d + 1) * 12)
        self.lib.orc_frames(C.byref(self.scene), np.ascontiguousarray(q, dtype=np.float64), out)
        return out.reshape(self.d + 1, 3, 4)

    def spheres(self, q):
        out = np.zeros(self.prob.n_spheres * 3)
        self.lib.orc_sphere_centres(C.byref(self.scene), np.ascontiguousarray(q, dtype=np.float64), out)
        return out.reshape(-1, 3)

    def obstacle(self, o, t):
        out = np.zeros(3)
        self.lib.orc_obstacle_pos(C.byref(self.scene), o, float(t), out)
        return out

    # checks ----------------------------------------------------------------
    def state_valid(self, x):
        m = C.c_double()
        ok = self.lib.orc_state_valid(C.byref(self.scene), np.ascontiguousarray(x, dtype=np.float64), C.byref(m))
        return bool(ok), m.value

    def check_states(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        M = x.shape[0]
        free = np.zeros(M, dtype=np.uint8)
        margin = np.zeros(M)
        self.lib.orc_check_states(C.byref(self.scene), M, x, free, margin)
        return free, margin

    def check_edges(self, xa, xb):
        xa = np.ascontiguousarray(xa, dtype=np.float64)
        xb = np.ascontiguousarray(xb, dtype=np.float64)
        E = xa.shape[0]
        free = np.zeros(E, dtype=np.uint8)
        fh = np.zeros(E, dtype=np.int32)
        n = np.zeros(E, dtype=np.int64)
        m = np.zeros(E)
        nr = np.zeros(E)
        self.lib.orc_check_edges(C.byref(self.scene), E, xa, xb, free, fh, n, m, nr)
        return dict(free=free, first_hit=fh, n=n, margin=m, n_real=nr)

    def edge_continuous(self, xa, xb):
        dm = C.c_double()
        ok = self.lib.orc_edge_continuous(C.byref(self.scene), np.ascontiguousarray(xa, dtype=np.float64),
                                          np.ascontiguousarray(xb, dtype=np.float64), C.byref(dm))
        return bool(ok), dm.value

    # metric ----------------------------------------------------------------

    def edge_continuous_pw(self, xa, xb):
        """Exact continuous check, obstacle trajectories cut at their waypoints."""
        m = C.c_double()
        ok = self.lib.orc_edge_continuous_pw(C.byref(self.scene), np.ascontiguousarray(xa, dtype=np.float64),
                                             np.ascontiguousarray(xb, dtype=np.float64), C.byref(m))
        return bool(ok), m.value
    def rho(self, sigma, x, xr):
        return self.lib.orc_rho(self.d, float(self.prob.v_max), int(sigma),
                                np.ascontiguousarray(x, dtype=np.float64), np.ascontiguousarray(xr, dtype=np.float64))

    def nearest(self, nodes, xq, sigma=1, metric=0, mask=None):
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        dist = C.c_double()
        amb = C.c_uint8()
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        idx = self.lib.orc_nearest(C.byref(self.scene), nodes.shape[0], nodes, m, int(sigma), int(metric),
                                   np.ascontiguousarray(xq, dtype=np.float64), C.byref(dist), C.byref(amb))
        return int(idx), dist.value, bool(amb.value)

    # allocation ------------------------------------------------------------
    def lower_bound(self):
        return self.lib.orc_lower_bound(C.byref(self.scene))

    def goal_grid(self):
        lo, hi = C.c_int64(), C.c_int64()
        self.lib.orc_goal_grid_range(C.byref(self.scene), C.byref(lo), C.byref(hi))
        n = max(hi.value - lo.value + 1, 0)
        free = np.zeros(max(n, 1), dtype=np.uint8)
        if n > 0:
            self.lib.orc_goal_grid(C.byref(self.scene), lo.value, hi.value, free)
        return lo.value, hi.value, free[:n]

    def validate_path(self, states, U, Cst, rel_tol=1e-5):
        states = np.ascontiguousarray(states, dtype=np.float64)
        msg = C.create_string_buffer(256)
        ok = self.lib.orc_validate_path(C.byref(self.scene), states.shape[0], states, float(U), float(Cst),
                                        float(rel_tol), msg, 256)
        return bool(ok), msg.value.decode()


def ir_partition(L, H, Ubar, dt, k_lo, k_hi, free, N, maxp=64):
    lib = _load()
    I = np.zeros(2 * N)
    npc = np.zeros(N, dtype=np.int32)
    pieces = np.zeros(N * maxp * 2)
    r = lib.orc_ir_partition(float(L), float(H), float(Ubar), float(dt), int(k_lo), int(k_hi),
                             np.ascontiguousarray(free, dtype=np.uint8), int(N), I, npc, pieces, int(maxp))
    assert r >= 0, "too many pieces"
    pieces = pieces.reshape(N, maxp, 2)
    return I.reshape(N, 2), [pieces[i, :npc[i]].copy() for i in range(N)]


def philox(ctr, key):
    lib = _load()
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
    return out


class Planner:
    """The oracle's lockstep planner for one problem."""

    def __init__(self, prob, problem_id: int = 0):
        self.lib = _load()
        self.prob = prob
        self.scene = make_scene(prob, problem_id)
        self.h = self.lib.orc_planner_create(C.byref(self.scene))
        self.d = prob.d
        self.N = prob.params.n_groups

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.orc_planner_destroy(self.h)
            self.h = None

    def info(self):
        out = np.zeros(16)
        self.lib.orc_planner_info(self.h, out)
        keys = ["U", "C", "inc_f", "inc_b", "first_iter", "L", "H", "k_lo", "k_hi", "iter", "overflow",
                "n_active", "total", "n_pools", "edge_checks", "bridge_checks"]
        return {k: out[i] for i, k in enumerate(keys)}

    def counts(self):
        c = np.zeros(1 + self.N, dtype=np.int64)
        self.lib.orc_planner_counts(self.h, c)
        return c

    def goal_free(self):
        inf = self.info()
        n = int(inf["k_hi"] - inf["k_lo"] + 1)
        out = np.zeros(max(n, 1), dtype=np.uint8)
        if n > 0:
            self.lib.orc_planner_goal_free(self.h, out)
        return out[:max(n, 0)]

    def partition(self, maxp=4096):
        I = np.zeros(2 * self.N)
        npc = np.zeros(self.N, dtype=np.int32)
        pieces = np.zeros(self.N * maxp * 2)
        self.lib.orc_planner_partition(self.h, I, npc, pieces, maxp)
        pieces = pieces.reshape(self.N, maxp, 2)
        return I.reshape(self.N, 2), [pieces[i, :npc[i]].copy() for i in range(self.N)]

    def slots(self):
        T = np.zeros(self.N)
        a = np.zeros(self.N, dtype=np.int32)
        g = np.zeros(self.N, dtype=np.uint32)
        k = np.zeros(self.N, dtype=np.int64)
        self.lib.orc_planner_slots(self.h, T, a, g, k)
        return T, a, g, k

    def sample(self, it, B=None):
        B = B or self.prob.params.batch
        d = self.d
        out = dict(dir=np.zeros(B, dtype=np.int8), flags=np.zeros(B, dtype=np.uint8),
                   grp=np.zeros(B, dtype=np.int32), T=np.zeros(B), qr=np.zeros(d * B), tr=np.zeros(B))
        self.lib.orc_planner_sample(self.h, it, B, out["dir"], out["flags"], out["grp"], out["T"], out["qr"],
                                    out["tr"])
        out["qr"] = out["qr"].reshape(d, B)
        return out

    def extend(self, s):
        B = s["dir"].shape[0]
        d = self.d
        o = dict(status=np.zeros(B, dtype=np.int8), parent=np.zeros(B, dtype=np.int32),
                 new_idx=np.zeros(B, dtype=np.int32), xnew=np.zeros((d + 1) * B),
                 bridge=np.zeros(B, dtype=np.int32), bridge_ok=np.zeros(B, dtype=np.uint8),
                 Up=np.zeros(B), Cp=np.zeros(B), amb=np.zeros(B, dtype=np.uint8),
                 edge_margin=np.zeros(B), bridge_margin=np.zeros(B))
        r = self.lib.orc_planner_extend(
            self.h, B, np.ascontiguousarray(s["dir"], dtype=np.int8), np.ascontiguousarray(s["flags"], dtype=np.uint8),
            np.ascontiguousarray(s["grp"], dtype=np.int32), np.ascontiguousarray(s["T"], dtype=np.float64),
            np.ascontiguousarray(np.asarray(s["qr"], dtype=np.float64).reshape(-1)),
            np.ascontiguousarray(s["tr"], dtype=np.float64),
            o["status"], o["parent"], o["new_idx"], o["xnew"], o["bridge"], o["bridge_ok"], o["Up"], o["Cp"],
            o["amb"], o["edge_margin"], o["bridge_margin"])
        o["xnew"] = o["xnew"].reshape(d + 1, B)
        o["improved"] = r
        return o

    def bridge(self, sigma, x, x_rootT):
        """Best-ranked bridge from x into the opposite set of the current trees:
        (global index or -1, arrival time, fragile flag)."""
        arr = C.c_double()
        amb = C.c_uint8()
        b = self.lib.orc_planner_bridge(self.h, int(sigma), np.ascontiguousarray(x, dtype=np.float64),
                                        float(x_rootT), C.byref(arr), C.byref(amb))
        return int(b), arr.value, bool(amb.value)

    def recycle(self, U):
        """A strict drop of U to the given value followed by the recycling
        update (Alg. 3), outside the extend step."""
        if self.lib.orc_planner_recycle(self.h, float(U)) != 0:
            raise ValueError("recycle: not a recycling planner or U not below the incumbent")

    def set_proposal(self, z, mix):
        self.lib.orc_planner_set_proposal(self.h, None if z is None else np.ascontiguousarray(z, dtype=np.float64),
                                          float(mix))

    def run(self, iters):
        return self.lib.orc_planner_run(self.h, int(iters))

    def path(self, max_n=1 << 16):
        st = np.zeros(max_n * (self.d + 1))
        n = self.lib.orc_planner_path(self.h, max_n, st)
        if n < 0:
            return None
        return st[: n * (self.d + 1)].reshape(n, self.d + 1)

    def export(self):
        inf = self.info()
        tot = int(inf["total"])
        x = np.zeros(tot * (self.d + 1))
        par = np.zeros(tot, dtype=np.int32)
        cost = np.zeros(tot)
        rootT = np.zeros(tot)
        self.lib.orc_planner_export(self.h, x, par, cost, rootT)
        return dict(x=x.reshape(tot, self.d + 1), parent=par, cost=cost, rootT=rootT, counts=self.counts())

    def import_state(self, counts, x, parent, cost, rootT, U, Cst, inc_f, inc_b, it, slots=None):
        if slots is None:
            sT = sa = sg = sk = None
        else:
            sT, sa, sg, sk = [np.ascontiguousarray(a) for a in slots]
            sT = sT.astype(np.float64)
            sa = sa.astype(np.int32)
            sg = sg.astype(np.uint32)
            sk = sk.astype(np.int64)
        self.lib.orc_planner_import(
            self.h, np.ascontiguousarray(counts, dtype=np.int64), np.ascontiguousarray(x, dtype=np.float64).reshape(-1),
            np.ascontiguousarray(parent, dtype=np.int32), np.ascontiguousarray(cost, dtype=np.float64),
            np.ascontiguousarray(rootT, dtype=np.float64), float(U), float(Cst), int(inc_f), int(inc_b), int(it),
            sT, sa, sg, sk)
