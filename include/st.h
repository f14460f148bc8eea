/*
 * st.h -- C ABI of the MI355X space-time extend engine (ST-pRRTC hot path).
 *
 * The library plans single-goal space-time motions among obstacles moving on
 * known trajectories with the two allocation policies of the paper
 * "ST-pRRTC: Parallel Space-Time RRT-C with Adaptive Goal-Time Forests":
 * interval root (Sec. IV-B, Alg. 2) and root recycling (Sec. V, Alg. 3), both
 * built on the extend step of Alg. 1.  Every step runs in hand-written HIP
 * kernels for gfx950; the host part only launches and reads results back.
 *
 * Conventions shared by every entry point
 *  - Return value: 0 = ok; positive = informational (ST_NO_SOLUTION,
 *    ST_TRIVIAL); negative = error, with a message from st_last_error().
 *    No exception crosses the ABI.
 *  - A space-time state is d+1 floats: the configuration q (d joint values
 *    or, for a translating robot, its position) followed by the time t.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller and only read
 *    during the call unless stated otherwise.
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.
 *    Calls that take a stream are asynchronous on it.
 *  - A problem handle is not thread-safe; distinct handles are independent.
 */
#ifndef ST_H
#define ST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ST_MAX_DOF 7
#define ST_MAX_SPHERES 128
#define ST_MAX_OBSTACLES 64
#define ST_MAX_WAYPOINTS 32
#define ST_MAX_GROUPS 128
#define ST_MAX_SELF_PAIRS 32
#define ST_MAX_BOXES 16

/* return codes */
#define ST_OK 0
#define ST_NO_SOLUTION 1   /* budget spent or start invalid: no incumbent */
#define ST_TRIVIAL 2       /* q_s = q_g, start free and arrival at 0 allowed */
#define ST_EINVAL (-1)     /* bad sizes, NaN, t_min > t_max, v_max <= 0, ... */
#define ST_ENOMEM (-2)
#define ST_EHIP (-3)       /* a HIP runtime call failed */
#define ST_ECAPACITY (-4)  /* no solution, and some insert was dropped because its tree pool was full */

/* robot kinds */
#define ST_ROBOT_TRANSLATE 0 /* sphere centre = (q0, q1[, q2]) + local offset (d = 2 or 3) */
#define ST_ROBOT_DH 1        /* serial chain, standard Denavit-Hartenberg */

/* allocation policies */
#define ST_INTERVAL_ROOT 0   /* Sec. IV-B, Alg. 2 */
#define ST_ROOT_RECYCLING 1  /* Sec. V, Alg. 3 */

/* node sets for st_nearest */
#define ST_SET_FORWARD (-1)       /* the shared forward tree rooted at (q_s, 0) */
#define ST_SET_ALL_BACKWARD (-2)  /* every active backward tree */
/* set >= 0 selects backward group `set` (interval root) or slot `set` (root recycling) */

/* metrics for st_nearest */
#define ST_METRIC_RHO 0      /* directed space-time distance, Eq. 7 */
#define ST_METRIC_CONFIG 1   /* configuration distance (root recycling, Sec. V) */

/* sample flags (st_samples.flags) */
#define ST_FLAG_SKIP 1       /* root or query sample rejected: the worker does nothing */
#define ST_FLAG_USE_NEW 2    /* backward worker uses the virtual root (q_g, T) as its source */
#define ST_FLAG_LEARNED 4    /* the sample came from the learned proposal */

/* extend status (st_extend_out.status) */
#define ST_STATUS_SKIPPED 0
#define ST_STATUS_TRAPPED 1  /* Alg. 1 returned TRAPPED */
#define ST_STATUS_ADVANCED 2 /* x_new appended */
#define ST_STATUS_DROPPED 3  /* advanced but the tree pool was full (see st_extend_batch) */

/* Planner parameters.  The paper fixes N = 64, 1024 configurations per batch,
 * p_new = 0.05, p_guided = 0.95 and dt = 0.02 s (Sec. VI); eta, the edge
 * resolution h and the capacities are not stated there. */
typedef struct st_params {
    int32_t variant;     /* ST_INTERVAL_ROOT or ST_ROOT_RECYCLING */
    int32_t n_groups;    /* N: groups (interval root) or slots (recycling), 1..ST_MAX_GROUPS */
    int32_t batch;       /* B: workers (samples) per iteration */
    double eta;          /* steering range (Alg. 1, Eq. 8) */
    double h;            /* edge discretisation step in the configuration metric */
    double dt;           /* environment time step: goal-grid spacing (Eq. 5) */
    double p_new;        /* probability of a fresh virtual root (Alg. 2) */
    double p_guided;     /* probability of sampling T from guided windows (Sec. IV-B) */
    int32_t cap_fwd;     /* forward-tree capacity (nodes) */
    int32_t cap_bwd;     /* capacity of each backward pool (one per group / slot) */
    uint32_t seed;       /* Philox4x32-10 key word 0 */
    uint32_t problem_id; /* Philox4x32-10 key word 1 */
    int32_t no_recycling;/* recycling variant: 1 keeps the initial roots, deactivation
                            only (the allocation ablation of Sec. VI); 0 recycles (Alg. 3) */
    int32_t obstacle_tile;/* obstacles per register tile of the collision kernels: 0 picks 4, 8
                            or 16 by the obstacle count; 4, 8 or 16 forces it (obstacles padded
                            with far, zero-radius ones to a multiple of it; decisions unchanged).
                            Problems of one batch that share a tile share kernel instances. */
} st_params;

/* Problem description (Sec. III): robot, configuration box C, start q_s,
 * goal q_g, arrival range [t_min, t_max] (horizon H = t_max), obstacles on
 * known piecewise-linear trajectories, speed limit v_max (Eq. 2).
 * All pointers are host memory, copied by st_problem_create. */
typedef struct st_problem_desc {
    int32_t dof;                   /* d, 1..ST_MAX_DOF */
    int32_t robot_kind;            /* ST_ROBOT_TRANSLATE or ST_ROBOT_DH */
    const double *dh;              /* [d][4]: a, alpha, d, theta0 (DH only, may be NULL otherwise) */
    int32_t n_spheres;             /* S, 1..ST_MAX_SPHERES */
    const int32_t *sphere_link;    /* [S]: 0 = base frame, l = frame after joint l */
    const double *spheres;         /* [S][4]: centre in the link frame, radius */
    const double *q_lo, *q_hi;     /* [d] configuration box C */
    const double *q_start, *q_goal;/* [d] */
    double t_min, t_max;           /* arrival range; H = t_max */
    double v_max;                  /* speed limit in the Euclidean configuration metric */
    int32_t n_obstacles;           /* O, 0..ST_MAX_OBSTACLES */
    int32_t max_waypoints;         /* row stride of waypoints, 1..ST_MAX_WAYPOINTS */
    const int32_t *n_waypoints;    /* [O], each 1..max_waypoints */
    const double *waypoints;       /* [O][max_waypoints][4]: t, x, y, z (times non-decreasing) */
    const double *obstacle_radius; /* [O] */
    st_params params;
    /* Static geometry of an arm (ST_ROBOT_DH only; zero counts switch it off).
     * Time-independent terms of the state test, after the sphere checker the
     * paper reuses (Sec. VI):
     *  - self collision: pair k = (la, lb), 0 <= la < lb <= d, tests every
     *    sphere of link la against every sphere of link lb (free iff at least
     *    r_s + r_s' apart); duplicates are ignored;
     *  - fixed oriented boxes: a sphere is free iff its centre is at least r_s
     *    from the closed box. */
    int32_t n_self_pairs;          /* 0..ST_MAX_SELF_PAIRS */
    const int32_t *self_pairs;     /* [n_self_pairs][2] link indices */
    int32_t n_boxes;               /* 0..ST_MAX_BOXES */
    const double *boxes;           /* [n_boxes][15]: centre (3), half extents (3, >= 0), then the
                                      three unit box axes in world coordinates, one per row
                                      (orthonormal to 1e-6) */
} st_problem_desc;

typedef struct st_problem st_problem;

/* Device SoA batch of samples (worker inputs, Alg. 2 / Alg. 3). B entries each. */
typedef struct st_samples {
    int8_t *dir;     /* 0 = forward (sigma = +1), 1 = backward (sigma = -1) */
    uint8_t *flags;  /* ST_FLAG_* */
    int32_t *grp;    /* group i (interval root) or slot (recycling) */
    float *T;        /* root time of the group sample (interval root) or slot root */
    float *qr;       /* [d][B] query configuration q_r */
    float *tr;       /* [B] query time t_r (Eq. 6; unused by recycling) */
} st_samples;

/* Device SoA results of one extend batch. B entries each. */
typedef struct st_extend_out {
    int8_t *status;    /* ST_STATUS_* */
    int32_t *parent;   /* parent of x_new (global node index), -1 if none */
    int32_t *new_idx;  /* global index of x_new, -1 if not inserted */
    float *xnew;       /* [d+1][B] steered state (valid when advanced) */
    int32_t *bridge;   /* best-ranked bridge target (global index), -1 if none */
    uint8_t *bridge_ok;/* 1 when that bridge is collision free */
    float *Up;         /* candidate arrival U' (inf when no valid bridge) */
    float *Cp;         /* candidate path length C' */
} st_extend_out;

typedef struct st_budget {
    int64_t max_iters;   /* > 0: stop after this many iterations */
    double max_ms;       /* > 0: stop after this much wall time */
    int32_t stop_at_first; /* 1: return as soon as a first solution exists */
    int32_t iters_per_sync;/* iterations launched between host checks (0 = 8) */
} st_budget;

/* Host result of st_plan; states is library-allocated, free with st_path_free. */
typedef struct st_path {
    int64_t n_states;
    int32_t dof;
    double *states;          /* [n_states][d+1]: (q_s, 0) ... (q_g, U) */
    double arrival;          /* U */
    double length;           /* C: configuration path length */
    int64_t iterations;
    int64_t first_solution_iter;
    double first_solution_ms;/* device time from the first iteration's launch to the end of the launches
                                (iters_per_sync iterations) that found the first incumbent; the start
                                check and the launch set-up (buffers, graph capture) come before it and
                                are not counted.  st_plan_sequence: the sum over its legs */
    double total_ms;         /* wall time of the call, set-up included */
} st_path;

/* Snapshot of the planner state (host). */
typedef struct st_info {
    double U, C;              /* incumbent (inf, inf when none) */
    int64_t inc_fwd, inc_bwd; /* incumbent endpoints (global node indices) */
    double L, H;              /* search domain [L, H], L = max(L_g, t_min) (Eq. 5) */
    int64_t k_lo, k_hi;       /* goal-grid indices */
    int64_t iter;
    int32_t overflow;         /* some insert was dropped for capacity */
    int32_t n_active;         /* active recycling slots */
    int64_t total_cap;        /* cap_fwd + N cap_bwd */
    int32_t n_pools;          /* 1 + N */
    int64_t first_iter;       /* iteration of the first incumbent, -1 if none */
    /* launch shape (the batch of many problems reads these at st_batch_create) */
    int32_t batch;            /* samples per iteration B */
    int32_t obstacle_tile;    /* obstacles per register tile of the collision kernels */
    int32_t lanes_extension, lanes_bridge, lanes_check; /* lanes per edge chunk (st_set_tuning) */
} st_info;

/* ---- lifecycle -------------------------------------------------------- */

/* Validate and copy the description, upload the scene, allocate the trees on
 * the current device, compute the goal grid valid(q_g, k dt) (Eq. 5) and the
 * initial allocation (interval-root partition or recycling roots).  The handle
 * owns all device memory.  Errors: ST_EINVAL, ST_ENOMEM, ST_EHIP.  Besides the
 * per-field limits, the scene staged per block must fit in 64 KB of LDS:
 * 32 B per obstacle (rounded up to the obstacle tile of 4, 8 or 16) and
 * trajectory segment (max_waypoints - 1, at least 1), 32 B per sphere, 64 B per
 * box, and 4 B per obstacle and waypoint when the obstacles' waypoint times
 * differ; a larger scene is ST_EINVAL (e.g. 64 obstacles with 16 waypoints fit,
 * 64 with 32 do not). */
int st_problem_create(const st_problem_desc *desc, st_problem **out);

/* Release the handle and its device memory.  Null-safe. */
void st_problem_destroy(st_problem *p);

/* Drop all nodes and the incumbent and re-initialise the trees and the
 * allocation (same scene).  Synchronous. */
int st_problem_reset(st_problem *p);

/* ---- collision (Sec. VI: obstacles interpolated at absolute times) ------ */

/* valid(q,t) for M states.  x: device [M][d+1]; free_out: device [M] (1 = free).
 * A state is free when q is inside C, 0 <= t <= H and every robot sphere is at
 * least r_s + r_o from every obstacle (touching is free), and, with static
 * geometry, the listed link pairs and the boxes are clear as well. */
int st_check_states(st_problem *p, int64_t M, const float *x, uint8_t *free_out, void *stream);

/* Discretised edge validity ("collision-checked along their interpolations",
 * Sec. IV-B).  xa, xb: device [E][d+1].  The edge is ordered by time, split
 * into n = max(1, ceil(max(D, v_max |dt|) / h)) steps and its n+1 states are
 * checked.  free_out: device [E]; first_hit: device [E] or NULL, receives the
 * least colliding state index in time order (-1 if free).  The result does not
 * depend on the order of the endpoints. */
int st_check_edges(st_problem *p, int64_t E, const float *xa, const float *xb, uint8_t *free_out,
                   int32_t *first_hit, void *stream);

/* st_check_edges for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * check and results, with the pipeline's work lists in a fixed device array
 * of the library instead of buffers it allocates, so the call allocates
 * nothing (host or device).  E <= ST_NOALLOC_MAX_EDGES, else ST_EINVAL.  The
 * array (about 8.6 MB) is held on every device the call runs on until the
 * process ends; all calls on one device share it, so calls that overlap on a
 * device (different streams or threads) race and must be serialised by the
 * caller.  Inputs and outputs as for st_check_edges.  Async on stream. */
#define ST_NOALLOC_MAX_EDGES 65536
int st_check_edges_noalloc(st_problem *p, int64_t E, const float *xa, const float *xb, uint8_t *free_out,
                           int32_t *first_hit, void *stream);

/* Exact continuous check of edges for a translating robot (ST_ROBOT_TRANSLATE):
 * the edge's time span is cut where an obstacle changes trajectory segment;
 * on each piece robot and obstacle move linearly and every sphere pair's
 * closest approach is taken in closed form, so no discretisation step is
 * involved (an alternative to the h-discretised check of Sec. IV-B for
 * disc-type scenes).  Free iff both endpoints lie in the box and the horizon
 * and every pair keeps distance >= r_s + r_o (touching is free).  xa, xb:
 * device [E][d+1]; free_out: device [E]; dmin_out: device [E] least pair
 * clearance (may be NULL).  EINVAL for arm robots.  Async on stream. */
int st_check_edges_continuous(st_problem *p, int64_t E, const float *xa, const float *xb, uint8_t *free_out,
                              float *dmin_out, void *stream);

/* ---- nearest node (Alg. 1, Eq. 7) -------------------------------------- */

/* For each of M queries xq (device [M][d+1]) find the node of `set` that
 * minimises the metric: ST_METRIC_RHO is rho_sigma of Eq. 7 (infinite unless
 * sigma (t_q - t_v) > 0 and D <= v_max sigma (t_q - t_v)); ST_METRIC_CONFIG is
 * the configuration distance.  Backward sets of interval root only contain
 * trees rooted below the incumbent U.  idx_out: device [M] (-1 when nothing is
 * admissible), dist_out: device [M] or NULL (rho or D; inf when -1).  Ties go
 * to the lowest node index. */
int st_nearest(st_problem *p, int32_t set, int32_t metric, int32_t sigma, int64_t M, const float *xq,
               int32_t *idx_out, float *dist_out, void *stream);

/* ---- batched extension (Alg. 1-3) --------------------------------------- */

/* Draw B worker samples for iteration `iter` with Philox4x32-10 keyed by
 * (seed, problem_id), counter (iter, worker, block, 0): direction alternating
 * as (worker + iter) mod 2; interval root: group, root time T from the group's
 * guided portions or uniform interval, the root check valid(q_g, T), q_r ~ U(C)
 * and t_r by Eq. 6 (empty interval rejected), and the p_new rule; root
 * recycling: the k-th backward worker takes active slot k mod n_active, q_r ~ U(C).
 * out: device SoA with B entries. */
int st_sample_batch(st_problem *p, int64_t iter, int64_t B, const st_samples *out, void *stream);

/* Run Alg. 1 for B workers against the trees as they are at entry (inserts of
 * this batch are not visible to it): nearest node, steering (interval root:
 * alpha = min(1, eta / rho); recycling: Eq. 8), the [0, H] and edge checks, the
 * insert (nodes of one pool are numbered in worker order; a virtual source is
 * materialised as a new tree root first), the best-ranked bridge into the
 * opposite set and its check, the candidate (U', C').  Capacity: the advanced
 * workers of a pool claim consecutive slots in worker order (two when a
 * virtual root is materialised), dropped claims included, as an atomic slot
 * counter hands them out; a worker whose claim ends past the pool's capacity
 * gets ST_STATUS_DROPPED (so the dropped workers of a pool are a suffix in
 * worker order), inserts nothing and takes no part in the incumbent update;
 * st_info.overflow is set.  Then the incumbent takes
 * the lexicographic minimum (U', C', worker) if it improves on (U, C), and on a
 * strict drop of U the allocation is updated (interval root: repartition and
 * deactivation of trees rooted at T >= U; recycling: deactivation and donor
 * replacement).  s, o: device SoA (o may have NULL members).  Async on stream. */
int st_extend_batch(st_problem *p, int64_t B, const st_samples *s, const st_extend_out *o, void *stream);

/* Sample + extend for `iters` iterations starting at the problem's iteration
 * counter, without host round trips.  Iterations after termination (interval
 * root: L >= min(H, U)) do nothing.  Async on stream. */
int st_iterate(st_problem *p, int64_t iters, void *stream);

/* Full planning loop (Alg. 2 / Alg. 3) within the budget; out receives the
 * incumbent path (host, library-allocated).  Returns ST_OK, ST_NO_SOLUTION or
 * ST_TRIVIAL; ST_ECAPACITY when the call ends without an incumbent and some
 * insert was dropped for capacity (the trees stopped growing; out holds no
 * states, its other fields are filled).  A path found despite dropped
 * inserts is ST_OK with st_info.overflow set.  Synchronous. */
int st_plan(st_problem *p, const st_budget *budget, st_path *out);

void st_path_free(st_path *path);

/* A goal sequence (Sec. III: q_g^1, ..., q_g^m visited in order), planned as
 * successive single-goal queries: query i starts at the previous goal with
 * local time 0, the obstacle trajectories shifted by the previous arrival
 * and the remaining horizon; only the last goal keeps the arrival range's
 * lower end.  desc gives the robot, the start, the obstacles, the horizon and
 * the parameters (desc->q_goal is ignored); goals: host [m][d].  Each query
 * gets the budget.  out: the whole path in absolute time (host,
 * library-allocated, st_path_free), arrival T_m and total length.  Returns
 * ST_OK or ST_NO_SOLUTION (some query failed; out holds no states).
 * Synchronous. */
int st_plan_sequence(const st_problem_desc *desc, int32_t m, const double *goals, const st_budget *budget,
                     st_path *out);

/* Goal sequences of many problems planned together (Sec. III, as
 * st_plan_sequence does for one): leg i of every problem that has an i-th goal
 * and has not failed is planned in one batch of many problems (st_batch_*),
 * each leg with the budget (applied to the whole batch of that leg), and the
 * legs are joined in absolute time.  descs: host [P]; m: host [P] goal
 * counts (>= 1); goals: host [P] pointers to host [m[k]][d_k] (desc->q_goal is
 * ignored); outs: host [P], library-allocated paths (free each with
 * st_path_free); rcs: host [P] per-problem result (ST_OK, ST_NO_SOLUTION
 * when some leg found no path or no horizon was left, ST_ECAPACITY).  Returns
 * ST_OK when every problem was processed, else the first error.
 * Synchronous. */
int st_plan_sequence_batch(const st_problem_desc *descs, int32_t P, const int32_t *m, const double *const *goals,
                           const st_budget *budget, st_path *outs, int32_t *rcs);

/* The current incumbent path of a problem (host, library-allocated; free with
 * st_path_free).  Returns ST_OK, ST_NO_SOLUTION, or ST_ECAPACITY as st_plan
 * does.  Synchronous. */
int st_path_get(st_problem *p, st_path *out);

/* ---- many problems per launch (an addition to the paper's method) --------- */

/* A batch runs one iteration of every member problem as one launch sequence:
 * each kernel of the pipeline is launched once for all members (once per
 * scene class for the two kernels specialised by robot kind, obstacle tile
 * and obstacle-time mode), one grid dimension selecting the member; `iters_per_launch`
 * iterations are captured in one HIP graph.  The batch borrows the handles:
 * they must outlive it and must not be iterated on their own while it exists.
 * Each member keeps its own parameters (samples per iteration, launch shapes
 * from st_set_tuning); changing them after st_batch_create has no effect on
 * the batch.  Members whose start state collides, or that are trivial, take no
 * part in the launches.  A member may draw at most 65535 samples per iteration
 * (ST_EINVAL otherwise).  Synchronous. */
typedef struct st_batch st_batch;
int st_batch_create(st_problem *const *problems, int32_t n, int32_t iters_per_launch, st_batch **out);
void st_batch_destroy(st_batch *b);
/* `iters` iterations of every member (rounded up to whole launches).  Async. */
int st_batch_iterate(st_batch *b, int64_t iters, void *stream);

/* Per-member results of st_batch_plan; arrays are host memory owned by the
 * caller, [n] each (any may be NULL). */
typedef struct st_batch_result {
    double *first_ms;      /* device time from the call's start to the end of the launch that found the
                              member's first solution; NaN if none, 0 if it existed before the call */
    int64_t *first_iter;   /* iteration of the first solution, -1 if none */
    double *arrival;       /* incumbent arrival U, inf if none */
    int64_t iterations;    /* out: iterations run by the call */
    double total_ms;       /* out: wall time of the call */
    int32_t n_solved;      /* out: members with an incumbent */
} st_batch_result;
/* Iterate every member within the budget (max_iters, max_ms; stop_at_first:
 * until every member has a solution; iters_per_sync: iterations between host
 * checks, rounded up to whole launches).  Synchronous. */
int st_batch_plan(st_batch *b, const st_budget *budget, st_batch_result *res);

/* ---- state I/O (tests) -------------------------------------------------- */

int st_get_info(st_problem *p, st_info *out);

/* Export / import the node pools as host arrays in global numbering (pool 0 is
 * the forward tree at [0, cap_fwd); pool 1+i at [cap_fwd + i cap_bwd, ...)):
 * counts [1+N], x [total][d+1], parent [total], cost [total], rootT [total].
 * Import also sets the incumbent and iteration and recomputes the allocation;
 * slot arrays (T, active, gen, grid index; [N] each) may be NULL for interval
 * root.  Synchronous. */
int st_tree_export(st_problem *p, int64_t *counts, float *x, int32_t *parent, float *cost, float *rootT);
int st_tree_import(st_problem *p, const int64_t *counts, const float *x, const int32_t *parent, const float *cost,
                   const float *rootT, double U, double C, int64_t inc_fwd, int64_t inc_bwd, int64_t iter,
                   const double *slot_T, const int32_t *slot_active, const uint32_t *slot_gen,
                   const int64_t *slot_k);
int st_slots_export(st_problem *p, double *slot_T, int32_t *slot_active, uint32_t *slot_gen, int64_t *slot_k);
/* goal grid valid(q_g, k dt) for k in [k_lo, k_hi] (host [k_hi - k_lo + 1]) */
int st_goal_grid_export(st_problem *p, uint8_t *free_out);
/* interval-root allocation: I [N][2], n_pieces [N], pieces [N][maxp][2] */
int st_partition_export(st_problem *p, double *I, int32_t *n_pieces, double *pieces, int32_t maxp);

/* ---- learned proposal (an addition to the paper's method) ---------------- */

/* The network proposes (q, t) query samples and goal arrival times; a worker
 * uses it with probability `mix` and the plain sampler otherwise, so the plain
 * sampler keeps full support.  Inputs per problem: core [16] = (q_s / pi,
 * q_g / pi, each padded to 7; t_min / 60, t_max / 60) and obstacle rows
 * [O][65] = 16 waypoints (t / 60, x, y, z; the last waypoint repeated) and the
 * radius, with a mask [O].  Output z [168] per problem: 8 mixture logits,
 * 8 x 8 means, 8 x 8 log standard deviations of the normalised state
 * (q / pi in slots 0..d-1, t / 60 in slot 7), 32 arrival-histogram logits over
 * [t_min, t_max].  Weights are a flat FP32 vector (We[65][64], be, W1[96][256],
 * b1, W2..W4 [256][256], b2..b4, W5[256][168], b5); GEMMs run on bfloat16
 * matrix cores with FP32 accumulation. */
#define ST_MLP_OUTPUTS 168
typedef struct st_mlp st_mlp;
/* Device buffers for batches of up to max_batch problems / examples. */
int st_mlp_create(int32_t max_batch, int32_t max_obstacles, st_mlp **out);
void st_mlp_destroy(st_mlp *net);
int64_t st_mlp_param_count(void);
/* host_in (may be NULL): new FP32 weights (Adam state reset); host_out (may be
 * NULL): receives the weights.  Synchronous. */
int st_mlp_params(st_mlp *net, const float *host_in, float *host_out);
/* Gradients of the last st_mlp_backward (host, param_count floats).  Synchronous. */
int st_mlp_grads(st_mlp *net, float *host_out);
/* Forward pass for M rows: core [M][16], obs [M][O][65], mask [M][O] (device);
 * z_out [M][168] (device, may be NULL).  Async on stream. */
int st_mlp_forward(st_mlp *net, int32_t M, int32_t O, const float *core, const float *obs, const float *mask,
                   float *z_out, void *stream);
/* Loss of the last forward pass: mixture negative log-likelihood of K path
 * states y [M][K][8] (mask ymask [M][K], dimension mask dmask [M][8]) plus the
 * cross-entropy of the arrival bin ubin [M]; loss_per_out [M] (device, may be
 * NULL); keeps dL/dz for st_mlp_backward (the loss is the mean over rows). */
int st_mlp_loss(st_mlp *net, int32_t K, const float *y, const float *ymask, const float *dmask, const int32_t *ubin,
                float *loss_per_out, void *stream);
int st_mlp_backward(st_mlp *net, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the FP32 weights. */
int st_mlp_adam(st_mlp *net, float lr, void *stream);
/* Install a problem's network output z (device [168]; NULL clears) and the
 * probability `mix` that a worker draws from it.  Async on stream. */
int st_proposal_set(st_problem *p, const float *z, float mix, void *stream);

/* ---- tuning ---------------------------------------------------------------- */

/* Launch shapes of the collision kernels: obstacles held in registers per
 * tile (4, 8 or 16, dividing the padded obstacle count; 0 keeps the current
 * value) and lanes per edge chunk for extension edges, bridge edges and
 * st_check_edges (powers of two up to 64; 0 keeps).  Results do not depend
 * on these.  Synchronous; drops captured iteration graphs. */
int st_set_tuning(st_problem *p, int32_t obstacle_tile, int32_t lanes_extension, int32_t lanes_bridge,
                  int32_t lanes_check);

/* Lanes per space-time state in the edge checks of the arm robots (1, 2 or 4:
 * the state's spheres are shared out among that many lanes, each composing
 * the kinematic chain itself; shorter dependent chains for launches too small
 * to fill the device, more instructions per state) for extension edges,
 * bridge edges and st_check_edges; -1 chooses by launch size (4 up to 256
 * edges, else 1; a batch counts the edges of all its members); 0 keeps.  A translating robot always uses
 * one lane per state.  Results do not depend on these.  Synchronous; drops
 * captured iteration graphs. */
int st_set_state_split(st_problem *p, int32_t split_extension, int32_t split_bridge, int32_t split_check);

/* Extension edges (at most ceil(sqrt(2) eta / h) + 1 states) are checked by a
 * flattened one-kernel path: a block of eight waves takes 4 x `edges_per_block`
 * consecutive edges (edges_per_block 1..8), lays their states end to end and
 * deals them to its waves in rounds of 64.
 * 0 selects the chunked path that bridges and st_check_edges use.  Results do
 * not depend on this.  Default 4.  In a batch (st_batch_create) a member on
 * the flattened path takes 8 (fewer, fuller blocks for many members).
 * Synchronous; drops captured graphs. */
int st_set_flat_extension(st_problem *p, int32_t edges_per_block);

/* ---- measurement ---------------------------------------------------------- */

#define ST_PROFILE_STAGES 9
/* Stage timing with HIP events recorded on the launch stream between the
 * pipeline stages (0 sample, 1 nearest node, 2 steer, 3 extension edge check,
 * 4 insert, 5 bridge selection, 6 bridge edge check, 7 publish and allocation,
 * 8 unused).  Enabling clears earlier marks.  Synchronous. */
int st_profile_enable(st_problem *p, int32_t enable);
/* ms[ST_PROFILE_STAGES]: summed milliseconds per stage since the last read;
 * marks (may be NULL): number of intervals per stage.  Synchronous; clears. */
int st_profile_read(st_problem *p, double *ms, int64_t *marks);
/* out[4]: extension edges decided, their states up to the first hit (all n+1
 * when free), bridge edges decided, their states.  Cumulative since create. */
int st_work_counters(st_problem *p, uint64_t *out);

/* Thread-local message for the last error on this thread ("" if none). */
const char *st_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ST_H */
