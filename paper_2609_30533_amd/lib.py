"""Thin ctypes binding of the C ABI in include/st.h.

Argument marshalling only: every step of the planner runs in the HIP kernels
of libstprrtc.so.  PyTorch supplies device memory (tensor.data_ptr()) and the
stream (torch.cuda.current_stream().cuda_stream).  If the library has not been
built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import scenes

_HERE = os.path.dirname(os.path.abspath(__file__))
# STPRRTC_LIBRARY may name another build of the same library (A/B timing of
# kernel variants); by default the in-tree build is loaded
LIB_PATH = os.environ.get("STPRRTC_LIBRARY") or os.path.join(_HERE, "_build", "libstprrtc.so")

ST_OK, ST_NO_SOLUTION, ST_TRIVIAL = 0, 1, 2
ST_ECAPACITY = -4
SET_FORWARD, SET_ALL_BACKWARD = -1, -2
METRIC_RHO, METRIC_CONFIG = 0, 1
FLAG_SKIP, FLAG_USE_NEW = 1, 2
STATUS_SKIPPED, STATUS_TRAPPED, STATUS_ADVANCED, STATUS_DROPPED = 0, 1, 2, 3


class StError(RuntimeError):
    pass


class Params(C.Structure):
    _fields_ = [("variant", C.c_int32), ("n_groups", C.c_int32), ("batch", C.c_int32),
                ("eta", C.c_double), ("h", C.c_double), ("dt", C.c_double),
                ("p_new", C.c_double), ("p_guided", C.c_double),
                ("cap_fwd", C.c_int32), ("cap_bwd", C.c_int32),
                ("seed", C.c_uint32), ("problem_id", C.c_uint32), ("no_recycling", C.c_int32),
                ("obstacle_tile", C.c_int32)]


class Desc(C.Structure):
    _fields_ = [("dof", C.c_int32), ("robot_kind", C.c_int32), ("dh", C.POINTER(C.c_double)),
                ("n_spheres", C.c_int32), ("sphere_link", C.POINTER(C.c_int32)), ("spheres", C.POINTER(C.c_double)),
                ("q_lo", C.POINTER(C.c_double)), ("q_hi", C.POINTER(C.c_double)),
                ("q_start", C.POINTER(C.c_double)), ("q_goal", C.POINTER(C.c_double)),
                ("t_min", C.c_double), ("t_max", C.c_double), ("v_max", C.c_double),
                ("n_obstacles", C.c_int32), ("max_waypoints", C.c_int32),
                ("n_waypoints", C.POINTER(C.c_int32)), ("waypoints", C.POINTER(C.c_double)),
                ("obstacle_radius", C.POINTER(C.c_double)), ("params", Params),
                ("n_self_pairs", C.c_int32), ("self_pairs", C.POINTER(C.c_int32)),
                ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_double))]


class Samples(C.Structure):
    _fields_ = [("dir", C.c_void_p), ("flags", C.c_void_p), ("grp", C.c_void_p), ("T", C.c_void_p),
                ("qr", C.c_void_p), ("tr", C.c_void_p)]


class ExtendOut(C.Structure):
    _fields_ = [("status", C.c_void_p), ("parent", C.c_void_p), ("new_idx", C.c_void_p), ("xnew", C.c_void_p),
                ("bridge", C.c_void_p), ("bridge_ok", C.c_void_p), ("Up", C.c_void_p), ("Cp", C.c_void_p)]


class Budget(C.Structure):
    _fields_ = [("max_iters", C.c_int64), ("max_ms", C.c_double), ("stop_at_first", C.c_int32),
                ("iters_per_sync", C.c_int32)]


class Path(C.Structure):
    _fields_ = [("n_states", C.c_int64), ("dof", C.c_int32), ("states", C.POINTER(C.c_double)),
                ("arrival", C.c_double), ("length", C.c_double), ("iterations", C.c_int64),
                ("first_solution_iter", C.c_int64), ("first_solution_ms", C.c_double), ("total_ms", C.c_double)]


class BatchResult(C.Structure):
    _fields_ = [("first_ms", C.c_void_p), ("first_iter", C.c_void_p), ("arrival", C.c_void_p),
                ("iterations", C.c_int64), ("total_ms", C.c_double), ("n_solved", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("U", C.c_double), ("C", C.c_double), ("inc_fwd", C.c_int64), ("inc_bwd", C.c_int64),
                ("L", C.c_double), ("H", C.c_double), ("k_lo", C.c_int64), ("k_hi", C.c_int64),
                ("iter", C.c_int64), ("overflow", C.c_int32), ("n_active", C.c_int32), ("total_cap", C.c_int64),
                ("n_pools", C.c_int32), ("first_iter", C.c_int64), ("batch", C.c_int32),
                ("obstacle_tile", C.c_int32), ("lanes_extension", C.c_int32), ("lanes_bridge", C.c_int32),
                ("lanes_check", C.c_int32)]


# Every symbol the header declares (used by the load test).
EXPORTS = [
    "st_problem_create", "st_problem_destroy", "st_problem_reset", "st_check_states", "st_check_edges",
    "st_check_edges_continuous",
    "st_nearest", "st_sample_batch", "st_extend_batch", "st_iterate", "st_plan", "st_path_free", "st_get_info",
    "st_tree_export", "st_tree_import", "st_slots_export", "st_goal_grid_export", "st_partition_export",
    "st_set_tuning", "st_set_state_split", "st_set_flat_extension", "st_profile_enable", "st_profile_read", "st_work_counters", "st_last_error",
    "st_mlp_create", "st_mlp_destroy", "st_mlp_param_count", "st_mlp_params", "st_mlp_grads", "st_mlp_forward",
    "st_mlp_loss", "st_mlp_backward", "st_mlp_adam", "st_proposal_set",
    "st_path_get", "st_plan_sequence", "st_batch_create", "st_batch_destroy", "st_batch_iterate", "st_batch_plan",
    "st_check_edges_noalloc", "st_plan_sequence_batch",
]
NOALLOC_MAX_EDGES = 65536
NO_INT_RESULT = ("st_problem_destroy", "st_path_free", "st_last_error", "st_mlp_destroy", "st_mlp_param_count",
                 "st_batch_destroy")
STAGES = ["sample", "nearest", "steer", "edge_check", "insert", "bridge_select", "bridge_check", "publish"]

_lib = None


def load():
    """Load the built library; raise if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise StError("libstprrtc.so is not built (run __graft_entry__.build()); there is no CPU fallback")
    # PyTorch ships its own HIP runtime with the same soname; loading it first
    # makes this library bind to that one runtime instead of a second copy.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    L.st_problem_create.argtypes = [C.POINTER(Desc), C.POINTER(vp)]
    L.st_problem_destroy.argtypes = [vp]
    L.st_problem_destroy.restype = None
    L.st_problem_reset.argtypes = [vp]
    L.st_check_states.argtypes = [vp, i64, vp, vp, vp]
    L.st_check_edges.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.st_check_edges_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.st_nearest.argtypes = [vp, i32, i32, i32, i64, vp, vp, vp, vp]
    L.st_sample_batch.argtypes = [vp, i64, i64, C.POINTER(Samples), vp]
    L.st_extend_batch.argtypes = [vp, i64, C.POINTER(Samples), C.POINTER(ExtendOut), vp]
    L.st_iterate.argtypes = [vp, i64, vp]
    L.st_plan.argtypes = [vp, C.POINTER(Budget), C.POINTER(Path)]
    L.st_path_free.argtypes = [C.POINTER(Path)]
    L.st_path_free.restype = None
    L.st_get_info.argtypes = [vp, C.POINTER(Info)]
    L.st_tree_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.st_tree_import.argtypes = [vp, vp, vp, vp, vp, vp, dbl, dbl, i64, i64, i64, vp, vp, vp, vp]
    L.st_slots_export.argtypes = [vp, vp, vp, vp, vp]
    L.st_goal_grid_export.argtypes = [vp, vp]
    L.st_partition_export.argtypes = [vp, vp, vp, vp, i32]
    L.st_set_tuning.argtypes = [vp, i32, i32, i32, i32]
    L.st_set_state_split.argtypes = [vp, i32, i32, i32]
    L.st_set_flat_extension.argtypes = [vp, i32]
    L.st_profile_enable.argtypes = [vp, i32]
    L.st_profile_read.argtypes = [vp, vp, vp]
    L.st_work_counters.argtypes = [vp, vp]
    L.st_last_error.argtypes = []
    L.st_last_error.restype = C.c_char_p
    L.st_path_get.argtypes = [vp, C.POINTER(Path)]
    L.st_plan_sequence.argtypes = [C.POINTER(Desc), i32, C.POINTER(C.c_double), C.POINTER(Budget), C.POINTER(Path)]
    L.st_check_edges_continuous.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.st_plan_sequence_batch.argtypes = [C.POINTER(Desc), i32, vp, vp, C.POINTER(Budget), C.POINTER(Path), vp]
    L.st_batch_create.argtypes = [C.POINTER(vp), i32, i32, C.POINTER(vp)]
    L.st_batch_destroy.argtypes = [vp]
    L.st_batch_destroy.restype = None
    L.st_batch_iterate.argtypes = [vp, i64, vp]
    L.st_batch_plan.argtypes = [vp, C.POINTER(Budget), C.POINTER(BatchResult)]
    L.st_mlp_create.argtypes = [i32, i32, C.POINTER(vp)]
    L.st_mlp_destroy.argtypes = [vp]
    L.st_mlp_destroy.restype = None
    L.st_mlp_param_count.argtypes = []
    L.st_mlp_param_count.restype = i64
    L.st_mlp_params.argtypes = [vp, vp, vp]
    L.st_mlp_grads.argtypes = [vp, vp]
    L.st_mlp_forward.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.st_mlp_loss.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.st_mlp_backward.argtypes = [vp, vp]
    L.st_mlp_adam.argtypes = [vp, C.c_float, vp]
    L.st_proposal_set.argtypes = [vp, vp, C.c_float, vp]
    for name in EXPORTS:
        if name not in NO_INT_RESULT:
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc, what, allow=()):
    if rc < 0 and rc not in allow:
        raise StError("%s failed (%d): %s" % (what, rc, load().st_last_error().decode()))
    return rc


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    """Device pointer of a contiguous torch tensor (None for None)."""
    if t is None:
        return None
    assert t.is_contiguous()
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_desc(prob: scenes.Problem, problem_id: int = 0):
    """st_problem_desc for a generated problem; returns (desc, arrays to keep alive)."""
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double if dt == np.float64 else C.c_int32))

    D = Desc()
    D.dof, D.robot_kind = prob.d, prob.kind
    D.dh = arr(prob.dh, np.float64)
    D.n_spheres = prob.n_spheres
    D.sphere_link = arr(prob.sphere_link, np.int32)
    D.spheres = arr(prob.sphere, np.float64)
    D.q_lo, D.q_hi = arr(prob.q_lo, np.float64), arr(prob.q_hi, np.float64)
    D.q_start, D.q_goal = arr(prob.q_start, np.float64), arr(prob.q_goal, np.float64)
    D.t_min, D.t_max, D.v_max = prob.t_min, prob.t_max, prob.v_max
    D.n_obstacles, D.max_waypoints = prob.n_obs, max(prob.w_max, 1)
    D.n_waypoints = arr(prob.n_wp, np.int32)
    D.waypoints = arr(prob.wp, np.float64)
    D.obstacle_radius = arr(prob.obs_r, np.float64)
    p = prob.params
    D.params = Params(p.variant, p.n_groups, p.batch, p.eta, p.h, p.dt, p.p_new, p.p_guided, p.cap_fwd,
                      p.cap_bwd, p.seed & 0xFFFFFFFF, problem_id & 0xFFFFFFFF,
                      1 if getattr(p, "no_recycling", 0) else 0, int(getattr(p, "obstacle_tile", 0)))
    pairs = np.asarray(getattr(prob, "self_pairs", np.zeros((0, 2))), dtype=np.int32).reshape(-1, 2)
    boxes = np.asarray(getattr(prob, "boxes", np.zeros((0, 15))), dtype=np.float64).reshape(-1, 15)
    D.n_self_pairs = len(pairs)
    D.self_pairs = arr(pairs, np.int32) if len(pairs) else None
    D.n_boxes = len(boxes)
    D.boxes = arr(boxes, np.float64) if len(boxes) else None
    return D, keep


def plan_sequence(prob: scenes.Problem, goals, max_iters=0, max_ms=0.0, stop_at_first=False, iters_per_sync=0,
                  problem_id: int = 0):
    """st_plan_sequence: visit goals [m][d] in order from prob's start."""
    L = load()
    D, keep = make_desc(prob, problem_id)
    g = np.ascontiguousarray(goals, dtype=np.float64)
    b = Budget(max_iters, max_ms, 1 if stop_at_first else 0, iters_per_sync)
    path = Path()
    rc = _check(L.st_plan_sequence(C.byref(D), int(g.shape[0]), g.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(b), C.byref(path)), "st_plan_sequence", allow=(ST_ECAPACITY,))
    try:
        n = path.n_states
        d = prob.d
        states = np.ctypeslib.as_array(path.states, shape=(n * (d + 1),)).reshape(n, d + 1).copy() if n > 0 else None
        return dict(rc=rc, states=states, U=path.arrival, C=path.length, iterations=path.iterations,
                    first_ms=path.first_solution_ms, total_ms=path.total_ms)
    finally:
        L.st_path_free(C.byref(path))
        del keep


def plan_sequence_batch(probs, goal_lists, max_iters=0, max_ms=0.0, stop_at_first=False, iters_per_sync=0,
                        problem_ids=None):
    """st_plan_sequence_batch: every problem visits its goals [m_k][d_k] in
    order; leg i of all problems runs as one batch.  Returns one dict per
    problem (rc, states in absolute time, U, C, iterations)."""
    L = load()
    P = len(probs)
    ids = problem_ids if problem_ids is not None else list(range(P))
    descs = (Desc * P)()
    keep = []
    for k, (p, pid) in enumerate(zip(probs, ids)):
        D, kp = make_desc(p, pid)
        descs[k] = D
        keep.append(kp)
    gl = [np.ascontiguousarray(g, dtype=np.float64) for g in goal_lists]
    m = np.array([g.shape[0] for g in gl], dtype=np.int32)
    gptr = (C.POINTER(C.c_double) * P)(*[g.ctypes.data_as(C.POINTER(C.c_double)) for g in gl])
    outs = (Path * P)()
    rcs = np.zeros(P, dtype=np.int32)
    b = Budget(max_iters, max_ms, 1 if stop_at_first else 0, iters_per_sync)
    _check(L.st_plan_sequence_batch(descs, P, _ptr(m), C.cast(gptr, C.c_void_p), C.byref(b), outs, _ptr(rcs)),
           "st_plan_sequence_batch")
    res = []
    try:
        for k in range(P):
            path = outs[k]
            n, d = path.n_states, probs[k].d
            states = np.ctypeslib.as_array(path.states, shape=(n * (d + 1),)).reshape(n, d + 1).copy() \
                if (n > 0 and rcs[k] == ST_OK) else None
            res.append(dict(rc=int(rcs[k]), states=states, U=path.arrival, C=path.length,
                            iterations=path.iterations))
    finally:
        for k in range(P):
            L.st_path_free(C.byref(outs[k]))
        del keep, gl
    return res


class Problem:
    """One planning problem on the current HIP device."""

    def __init__(self, prob: scenes.Problem, problem_id: int = 0):
        self.L = load()
        self.prob = prob
        self.d = prob.d
        self.N = prob.params.n_groups
        D, keep = make_desc(prob, problem_id)
        h = C.c_void_p()
        _check(self.L.st_problem_create(C.byref(D), C.byref(h)), "st_problem_create")
        self.h = h
        del keep

    def close(self):
        if getattr(self, "h", None):
            self.L.st_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- collision ----------------------------------------------------------
    def check_states(self, x, out=None, stream=None):
        import torch
        M = x.shape[0]
        out = out if out is not None else torch.empty(M, dtype=torch.uint8, device=x.device)
        _check(self.L.st_check_states(self.h, M, _dptr(x), _dptr(out), _stream(stream)), "st_check_states")
        return out

    def check_edges(self, xa, xb, first_hit=True, stream=None):
        import torch
        E = xa.shape[0]
        free = torch.empty(E, dtype=torch.uint8, device=xa.device)
        fh = torch.empty(E, dtype=torch.int32, device=xa.device) if first_hit else None
        _check(self.L.st_check_edges(self.h, E, _dptr(xa), _dptr(xb), _dptr(free), _dptr(fh), _stream(stream)),
               "st_check_edges")
        return free, fh

    def check_edges_noalloc(self, xa, xb, free, first_hit=None, stream=None):
        """st_check_edges_noalloc into caller-provided outputs (E <= NOALLOC_MAX_EDGES)."""
        E = xa.shape[0]
        _check(self.L.st_check_edges_noalloc(self.h, E, _dptr(xa), _dptr(xb), _dptr(free), _dptr(first_hit),
                                             _stream(stream)), "st_check_edges_noalloc")
        return free, first_hit

    def check_edges_continuous(self, xa, xb, stream=None):
        """Exact continuous check (translating robots): (free, least clearance)."""
        import torch
        E = xa.shape[0]
        free = torch.empty(E, dtype=torch.uint8, device=xa.device)
        dmin = torch.empty(E, dtype=torch.float32, device=xa.device)
        _check(self.L.st_check_edges_continuous(self.h, E, _dptr(xa), _dptr(xb), _dptr(free), _dptr(dmin),
                                                _stream(stream)), "st_check_edges_continuous")
        return free, dmin

    # ---- nearest ------------------------------------------------------------
    def nearest(self, xq, set_id=SET_FORWARD, metric=METRIC_RHO, sigma=1, stream=None):
        import torch
        M = xq.shape[0]
        idx = torch.empty(M, dtype=torch.int32, device=xq.device)
        dist = torch.empty(M, dtype=torch.float32, device=xq.device)
        _check(self.L.st_nearest(self.h, set_id, metric, sigma, M, _dptr(xq), _dptr(idx), _dptr(dist),
                                 _stream(stream)), "st_nearest")
        return idx, dist

    # ---- batches ------------------------------------------------------------
    def alloc_samples(self, B, device="cuda"):
        import torch
        return dict(dir=torch.zeros(B, dtype=torch.int8, device=device),
                    flags=torch.zeros(B, dtype=torch.uint8, device=device),
                    grp=torch.zeros(B, dtype=torch.int32, device=device),
                    T=torch.zeros(B, dtype=torch.float32, device=device),
                    qr=torch.zeros(self.d, B, dtype=torch.float32, device=device),
                    tr=torch.zeros(B, dtype=torch.float32, device=device))

    @staticmethod
    def _samples_struct(s):
        return Samples(*[_dptr(s[k]) for k in ("dir", "flags", "grp", "T", "qr", "tr")])

    def sample(self, it, B=None, stream=None):
        B = B or self.prob.params.batch
        s = self.alloc_samples(B)
        S = self._samples_struct(s)
        _check(self.L.st_sample_batch(self.h, it, B, C.byref(S), _stream(stream)), "st_sample_batch")
        return s

    def extend(self, s, stream=None):
        import torch
        B = s["dir"].shape[0]
        dev = s["dir"].device
        o = dict(status=torch.zeros(B, dtype=torch.int8, device=dev),
                 parent=torch.zeros(B, dtype=torch.int32, device=dev),
                 new_idx=torch.zeros(B, dtype=torch.int32, device=dev),
                 xnew=torch.zeros(self.d + 1, B, dtype=torch.float32, device=dev),
                 bridge=torch.zeros(B, dtype=torch.int32, device=dev),
                 bridge_ok=torch.zeros(B, dtype=torch.uint8, device=dev),
                 Up=torch.zeros(B, dtype=torch.float32, device=dev),
                 Cp=torch.zeros(B, dtype=torch.float32, device=dev))
        S = self._samples_struct(s)
        O = ExtendOut(*[_dptr(o[k]) for k in ("status", "parent", "new_idx", "xnew", "bridge", "bridge_ok", "Up",
                                              "Cp")])
        _check(self.L.st_extend_batch(self.h, B, C.byref(S), C.byref(O), _stream(stream)), "st_extend_batch")
        return o

    def iterate(self, iters, stream=None):
        _check(self.L.st_iterate(self.h, iters, _stream(stream)), "st_iterate")

    def plan(self, max_iters=0, max_ms=0.0, stop_at_first=False, iters_per_sync=0):
        b = Budget(max_iters, max_ms, 1 if stop_at_first else 0, iters_per_sync)
        path = Path()
        # a plan that ends without a path after dropping inserts for capacity
        # is a result (rc = ST_ECAPACITY, no states), not an exception
        rc = _check(self.L.st_plan(self.h, C.byref(b), C.byref(path)), "st_plan", allow=(ST_ECAPACITY,))
        return self._path_dict(rc, path)

    def path(self):
        """The current incumbent path (st_path_get)."""
        path = Path()
        rc = _check(self.L.st_path_get(self.h, C.byref(path)), "st_path_get", allow=(ST_ECAPACITY,))
        return self._path_dict(rc, path)

    def _path_dict(self, rc, path):
        try:
            n = path.n_states
            states = np.ctypeslib.as_array(path.states, shape=(n * (self.d + 1),)).reshape(n, self.d + 1).copy() \
                if n > 0 else None
            res = dict(rc=rc, states=states, U=path.arrival, C=path.length, iterations=path.iterations,
                       first_iter=path.first_solution_iter, first_ms=path.first_solution_ms, total_ms=path.total_ms)
        finally:
            self.L.st_path_free(C.byref(path))
        return res

    def reset(self):
        _check(self.L.st_problem_reset(self.h), "st_problem_reset")

    # ---- state I/O ----------------------------------------------------------
    def info(self):
        inf = Info()
        _check(self.L.st_get_info(self.h, C.byref(inf)), "st_get_info")
        return {k: getattr(inf, k) for k, _ in Info._fields_}

    def export(self):
        inf = self.info()
        tot = inf["total_cap"]
        counts = np.zeros(1 + self.N, dtype=np.int64)
        x = np.zeros((tot, self.d + 1), dtype=np.float32)
        par = np.zeros(tot, dtype=np.int32)
        cost = np.zeros(tot, dtype=np.float32)
        rootT = np.zeros(tot, dtype=np.float32)
        _check(self.L.st_tree_export(self.h, _ptr(counts), _ptr(x), _ptr(par), _ptr(cost), _ptr(rootT)),
               "st_tree_export")
        return dict(counts=counts, x=x, parent=par, cost=cost, rootT=rootT)

    def import_state(self, counts, x, parent, cost, rootT, U, Cst, inc_f, inc_b, it, slots=None):
        counts = np.ascontiguousarray(counts, dtype=np.int64)
        x = np.ascontiguousarray(x, dtype=np.float32)
        parent = np.ascontiguousarray(parent, dtype=np.int32)
        cost = np.ascontiguousarray(cost, dtype=np.float32)
        rootT = np.ascontiguousarray(rootT, dtype=np.float32)
        if slots is not None:
            sT = np.ascontiguousarray(slots[0], dtype=np.float64)
            sa = np.ascontiguousarray(slots[1], dtype=np.int32)
            sg = np.ascontiguousarray(slots[2], dtype=np.uint32)
            sk = np.ascontiguousarray(slots[3], dtype=np.int64)
            sp = [_ptr(sT), _ptr(sa), _ptr(sg), _ptr(sk)]
        else:
            sp = [None] * 4
        _check(self.L.st_tree_import(self.h, _ptr(counts), _ptr(x), _ptr(parent), _ptr(cost), _ptr(rootT), float(U),
                                     float(Cst), int(inc_f), int(inc_b), int(it), *sp), "st_tree_import")

    def set_tuning(self, obstacle_tile=0, lanes_extension=0, lanes_bridge=0, lanes_check=0):
        _check(self.L.st_set_tuning(self.h, obstacle_tile, lanes_extension, lanes_bridge, lanes_check),
               "st_set_tuning")

    def set_state_split(self, extension=0, bridge=0, check=0):
        """Lanes per state (1, 2, 4; -1 by launch size; 0 keeps)."""
        _check(self.L.st_set_state_split(self.h, extension, bridge, check), "st_set_state_split")

    def set_flat_extension(self, edges_per_block):
        """Extension edges per block of the flattened path (0: chunked path)."""
        _check(self.L.st_set_flat_extension(self.h, int(edges_per_block)), "st_set_flat_extension")

    def set_proposal(self, z=None, mix=0.5, stream=None):
        """Install the network output z (device tensor [168]) for this problem."""
        _check(self.L.st_proposal_set(self.h, _dptr(z), float(mix if z is not None else 0.0), _stream(stream)),
               "st_proposal_set")

    def profile(self, enable=True):
        _check(self.L.st_profile_enable(self.h, 1 if enable else 0), "st_profile_enable")

    def profile_read(self):
        ms = np.zeros(9)
        marks = np.zeros(9, dtype=np.int64)
        _check(self.L.st_profile_read(self.h, _ptr(ms), _ptr(marks)), "st_profile_read")
        return {name: (float(ms[i]), int(marks[i])) for i, name in enumerate(STAGES)}

    def work_counters(self):
        out = np.zeros(4, dtype=np.uint64)
        _check(self.L.st_work_counters(self.h, _ptr(out)), "st_work_counters")
        return dict(edges=int(out[0]), edge_states=int(out[1]), bridges=int(out[2]), bridge_states=int(out[3]))

    def slots(self):
        T = np.zeros(self.N)
        a = np.zeros(self.N, dtype=np.int32)
        g = np.zeros(self.N, dtype=np.uint32)
        k = np.zeros(self.N, dtype=np.int64)
        _check(self.L.st_slots_export(self.h, _ptr(T), _ptr(a), _ptr(g), _ptr(k)), "st_slots_export")
        return T, a, g, k

    def goal_free(self):
        inf = self.info()
        n = inf["k_hi"] - inf["k_lo"] + 1
        out = np.zeros(max(n, 1), dtype=np.uint8)
        _check(self.L.st_goal_grid_export(self.h, _ptr(out)), "st_goal_grid_export")
        return out[:max(n, 0)]

    def partition(self, maxp=4096):
        I = np.zeros(2 * self.N)
        npc = np.zeros(self.N, dtype=np.int32)
        pieces = np.zeros(self.N * maxp * 2)
        _check(self.L.st_partition_export(self.h, _ptr(I), _ptr(npc), _ptr(pieces), maxp), "st_partition_export")
        pieces = pieces.reshape(self.N, maxp, 2)
        return I.reshape(self.N, 2), [pieces[i, :npc[i]].copy() for i in range(self.N)]


class Mlp:
    """The proposal network on the device (st_mlp_*)."""

    def __init__(self, max_batch, max_obstacles=32):
        self.L = load()
        h = C.c_void_p()
        _check(self.L.st_mlp_create(max_batch, max_obstacles, C.byref(h)), "st_mlp_create")
        self.h = h
        self.n_params = int(self.L.st_mlp_param_count())

    def close(self):
        if getattr(self, "h", None):
            self.L.st_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.size == self.n_params
        _check(self.L.st_mlp_params(self.h, _ptr(flat), None), "st_mlp_params")

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(self.L.st_mlp_params(self.h, None, _ptr(out)), "st_mlp_params")
        return out

    def grads(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(self.L.st_mlp_grads(self.h, _ptr(out)), "st_mlp_grads")
        return out

    def forward(self, core, obs, mask, z_out=None, stream=None):
        import torch
        M, O = obs.shape[0], obs.shape[1]
        z = z_out if z_out is not None else torch.empty(M, ST_MLP_OUTPUTS, dtype=torch.float32, device=core.device)
        _check(self.L.st_mlp_forward(self.h, M, O, _dptr(core), _dptr(obs), _dptr(mask), _dptr(z), _stream(stream)),
               "st_mlp_forward")
        return z

    def loss(self, y, ymask, dmask, ubin, stream=None):
        import torch
        M, K = y.shape[0], y.shape[1]
        per = torch.empty(M, dtype=torch.float32, device=y.device)
        _check(self.L.st_mlp_loss(self.h, K, _dptr(y), _dptr(ymask), _dptr(dmask), _dptr(ubin), _dptr(per),
                                  _stream(stream)), "st_mlp_loss")
        return per

    def backward(self, stream=None):
        _check(self.L.st_mlp_backward(self.h, _stream(stream)), "st_mlp_backward")

    def adam(self, lr, stream=None):
        _check(self.L.st_mlp_adam(self.h, float(lr), _stream(stream)), "st_mlp_adam")


ST_MLP_OUTPUTS = 168


class Batch:
    """Many problems per launch sequence (st_batch_*).  Keeps the Problem
    objects alive for its own lifetime."""

    def __init__(self, problems, iters_per_launch=4):
        self.L = load()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p.h for p in self.problems])
        h = C.c_void_p()
        _check(self.L.st_batch_create(arr, len(self.problems), int(iters_per_launch), C.byref(h)), "st_batch_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.st_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, iters, stream=None):
        _check(self.L.st_batch_iterate(self.h, int(iters), _stream(stream)), "st_batch_iterate")

    def plan(self, max_iters=0, max_ms=0.0, stop_at_first=False, iters_per_sync=0):
        n = len(self.problems)
        first_ms = np.zeros(n)
        first_iter = np.zeros(n, dtype=np.int64)
        arrival = np.zeros(n)
        r = BatchResult(first_ms.ctypes.data, first_iter.ctypes.data, arrival.ctypes.data, 0, 0.0, 0)
        b = Budget(max_iters, max_ms, 1 if stop_at_first else 0, iters_per_sync)
        _check(self.L.st_batch_plan(self.h, C.byref(b), C.byref(r)), "st_batch_plan")
        return dict(first_ms=first_ms, first_iter=first_iter, U=arrival, iterations=r.iterations,
                    total_ms=r.total_ms, n_solved=r.n_solved)
