// st_internal.hpp -- host-side problem object, device planner state and the
// kernel launchers shared by the translation units of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/st.h"
#include "st_device.hpp"

namespace st {

void set_error(const char *fmt, ...);

#define ST_HIP(call)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) {                                                                          \
            ::st::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return ST_EHIP;                                                                              \
        }                                                                                                \
    } while (0)

constexpr int kMaxGroups = ST_MAX_GROUPS;
constexpr int kMaxPools = kMaxGroups + 1;

// Planner state that lives in device memory (one record per problem).
struct PlanDev {
    float U, C;               // incumbent (arrival first, length breaks ties)
    int32_t inc_f, inc_b;     // incumbent endpoints (global node indices)
    int32_t improved;         // last batch: 0 none, 1 equal-U improvement, 2 strict drop of U
    int32_t done;             // interval root: L >= min(H, U)
    int32_t first_iter;       // iteration of the first incumbent (-1)
    int32_t overflow;         // an insert was dropped for capacity
    int32_t iter;             // iterations run so far
    int32_t n_active;         // recycling: active slots
    double Ubar;              // interval root: min(H, U)
    double G;                 // interval root: guided length below Ubar
    int32_t jstar;            // interval root: windows starting below Ubar
    int32_t pad0;
    float U_snap;             // U at the start of the current batch
    int32_t pad1;
    int32_t count[kMaxPools];       // nodes per pool
    int32_t count_snap[kMaxPools];  // nodes per pool at the start of the current batch
    float minRootT[kMaxGroups];     // interval root: earliest root time of the group's trees
    float slotT[kMaxGroups];        // recycling: root time per slot (inf when empty)
    int32_t slot_active[kMaxGroups];
    uint32_t slot_gen[kMaxGroups];
    int32_t slotK[kMaxGroups];      // goal-grid index of the slot's root
    int32_t active_list[kMaxGroups];
    // work counters: [0] extension edges decided, [1] their states up to the
    // first hit (n+1 when free), [2] bridge edges decided, [3] their states
    unsigned long long work[4];
    // learned proposal: probability of a learned draw, cumulative mixture
    // weights, means and standard deviations (normalised), cumulative
    // arrival-histogram weights
    float prop_mix;
    float prop_wcum[8];
    float prop_mu[64];
    float prop_sd[64];
    float prop_hcum[32];
};

// Node pools in device memory, SoA.
struct TreeDev {
    float *x;          // [d+1][total]
    int32_t *parent;   // [total]
    float *cost;       // [total]
    float *rootT;      // [total]
    int64_t total;
    int32_t cap_fwd, cap_bwd, n_pools, d;
};

__host__ __device__ inline int64_t pool_base(const TreeDev &t, int p) {
    return p == 0 ? 0 : (int64_t)t.cap_fwd + (int64_t)(p - 1) * t.cap_bwd;
}
__host__ __device__ inline int32_t pool_cap(const TreeDev &t, int p) { return p == 0 ? t.cap_fwd : t.cap_bwd; }

// Interval-root guided windows (merged, clipped to [L, H]).
struct WindowsDev {
    const double *lo, *hi, *cum;  // cum[j] = total length of windows 0..j-1
    int32_t nw;
    int32_t pad;
    double L, H, dt;
    int32_t N;
    int32_t k_lo, k_hi;
    const uint8_t *gfree;         // goal grid, [k_hi - k_lo + 1]
};

// Edge-check pipeline: hit[e] holds kNoHit until a colliding state is found;
// the rank counters sit kCntStride ints (128 bytes) apart.
constexpr int32_t kNoHit = 0x7fffffff;
constexpr int kBcntBridge = 128;  // bridge bucket counters (own cache lines)
constexpr int kBcntSize = 160;
constexpr int kCntStride = 32;

// Work buffers of the edge-check pipeline (capacity cap edges).
struct EdgeBufs {
    int64_t cap = 0;
    int32_t mmax = 0;           // work items per edge at most (<= 16)
    int32_t *n = nullptr;       // [cap] state count, -1 for skipped edges
    int32_t *hit = nullptr;     // [cap] least colliding state index found
    int2 *items = nullptr;      // [mmax][cap] (edge, rank)
    int32_t *cnt = nullptr;     // items per rank list, rank r at [32 r]
};

// One edge-check launch: the edges, their buffers and the grid sizes.
struct EdgeArgs {
    SceneDev sc;
    EdgeBufs eb;
    const float *xa, *xb;       // [E][d+1]
    const uint8_t *valid;       // [E] or null (all valid)
    uint8_t *free_out;          // [E]
    int32_t *first_hit;         // [E] or null
    unsigned long long *work;   // two work counters or null
    int64_t E;
    int32_t lpe_shift;          // lanes per chunk = 1 << lpe_shift
    int32_t split_shift;        // lanes per state = 1 << split_shift
    int32_t nb_edge;            // blocks of the per-edge kernels
    int32_t nb_items;           // blocks of the item kernel
    int32_t flat;               // > 0: short edges, flattened one-kernel path, this many per block
    int32_t skip_finish;        // 1: the consumer of the results does the finish step itself
};

// Per-batch work buffers (capacity Bcap workers).
struct Work {
    int64_t Bcap;
    // samples (owned copy used by st_iterate)
    int8_t *dir;
    uint8_t *flags;
    int32_t *grp;
    float *T, *qr, *tr;
    // extension
    unsigned long long *nn_key;  // [B] packed (distance bits, node index)
    int32_t *tiles;              // [4 * max_tiles]: set, first, count, sigma (st_nearest)
    int32_t *n_tiles;            // [2]
    // query buckets: the workers of each node set, set s at [s][Bcap]; their
    // counters at bcnt[s] (nearest-node sets = pools) and bcnt[kBcntBridge + s]
    // (bridge sets: 0 forward new nodes, 1 backward new nodes)
    int32_t *bcnt;
    int32_t *border_nn;          // [kMaxPools][Bcap]
    int32_t *border_br;          // [2][Bcap]
    float *xn, *xnew;            // [B][d+1]
    uint8_t *edge_valid, *edge_free;
    int32_t *first_hit;          // [B] scratch for the edge checks
    int8_t *status;
    int32_t *parent, *new_idx;
    float *cost_new, *rootT_new;
    // bridges
    unsigned long long *br_key;  // [B][nch]: bridge query (in bucket order) x node slice
    int32_t *br_idx;             // [B][nch]
    int32_t *bridge;
    float *xb;                   // [B][d+1]
    uint8_t *br_valid, *br_free;
    float *Up, *Cp;
};

}  // namespace st

struct st_problem {
    int device = 0;
    st_params prm{};
    int d = 0, kind = 0, S = 0, O = 0;
    std::vector<double> q_lo, q_hi, q_s, q_g;
    double t_min = 0, t_max = 0, v_max = 0, Lg = 0, L = 0;
    st::SceneDev sc{};
    float4 *d_sph = nullptr;
    float *d_ro = nullptr;     // obstacle radii [O_pad]
    float4 *d_seg = nullptr;
    float4 *d_goal = nullptr;  // sphere centres at q_g
    float *d_obs_r = nullptr;  // obstacle radii
    float4 *d_box = nullptr;   // static boxes, 4 rows each
    float *d_segt = nullptr;
    // goal grid and windows
    int64_t k_lo = 0, k_hi = -1;
    uint8_t *d_gfree = nullptr;
    std::vector<uint8_t> h_gfree;
    std::vector<double> h_wlo, h_whi, h_wcum;
    double *d_wlo = nullptr, *d_whi = nullptr, *d_wcum = nullptr;
    st::WindowsDev win{};
    // trees and planner state
    st::TreeDev tree{};
    st::PlanDev *d_plan = nullptr;
    st::Work work{};
    st::EdgeBufs ebufs{};      // planner edge checks (referenced by captured graphs)
    st::EdgeBufs ebufs_api{};  // st_check_edges
    int64_t iter = 0;
    int nch = 16;  // node chunks per query tile in scans
    // captured iterations: [0] one iteration, [1] four iterations
    bool use_graphs = true;
    // lanes per edge chunk (log2) for extension, bridge and st_check_edges launches
    int tune_ext = 5, tune_br = 4, tune_api = 5;
    // lanes per state (log2) for the same three launches; -1 chooses by size
    int split_ext = -1, split_br = -1, split_api = -1;
    // extension edges per block of the flattened path (0: chunked item path)
    int flat_ext = 4;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int64_t graph_B = 0;
    hipStream_t cap_stream = nullptr;
    // optional stage timing with HIP events (stage id per recorded event)
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_stage;
    size_t prof_used = 0;
};

namespace st {

// ---- collision ------------------------------------------------------------
size_t scene_lds_bytes(const SceneDev &sc);
// Exact continuous edge check (translating robots); dmin_out may be null.
hipError_t launch_check_edges_continuous(const SceneDev &sc, int64_t E, const float *xa, const float *xb,
                                         uint8_t *free_out, float *dmin_out, hipStream_t s);
// World centres (x, y, z, |c|^2) of the robot's spheres at q_g.
hipError_t launch_goal_centers(const SceneDev &sc, float4 *out);
hipError_t launch_check_states(const SceneDev &sc, int64_t M, const float *x, uint8_t *free_out, hipStream_t s);
int edge_bufs_reserve(EdgeBufs &eb, int64_t E);
void edge_bufs_free(EdgeBufs &eb);
// Lanes per chunk = 1 << lpe_shift (1..64).  first_hit and work may be null.
hipError_t launch_check_edges(const SceneDev &sc, const EdgeBufs &eb, int64_t E, const float *xa, const float *xb,
                              const uint8_t *valid, uint8_t *free_out, int32_t *first_hit, int lpe_shift,
                              hipStream_t s, unsigned long long *work = nullptr, int split_shift = 0);
// Lanes per state (log2) for a launch of E edges: explicit, or by size (only
// a few hundred edges leave most SIMDs idle, where shorter chains pay).
inline int split_for(int setting, int64_t E) {
    if (setting >= 0) return setting;
    return E <= 256 ? 2 : 0;
}
// Threads of an insertion block (one block per pool, four workers per thread
// and pass): whole waves, enough for one pass over B workers, at most 1024.
inline int insert_threads(int64_t B) {
    const int64_t t = ((B + 3) / 4 + 63) / 64 * 64;
    return (int)(t < 64 ? 64 : (t > 1024 ? 1024 : t));
}
// Record of one edge launch; the item kernel gets at least min_item_blocks blocks.
EdgeArgs edge_args(const SceneDev &sc, const EdgeBufs &eb, int64_t E, const float *xa, const float *xb,
                   const uint8_t *valid, uint8_t *free_out, int32_t *first_hit, int lpe_shift,
                   unsigned long long *work, int min_item_blocks, int split_shift);
hipError_t launch_edge_args(const EdgeArgs &a, hipStream_t s);
// The item kernel alone, for edges whose records (state count, least hit)
// and work items another kernel has written (the bridge check).
hipError_t launch_edge_items(const EdgeArgs &a, hipStream_t s);
// The same pipeline for P problems at once (records in device memory); the
// item kernel runs once per scene class over its member records.
hipError_t launch_edge_plan_multi(const EdgeArgs *d_args, int P, int max_nb_edge, hipStream_t s);
hipError_t launch_edge_items_multi(const SceneDev &cls, int split_shift, const EdgeArgs *d_args,
                                   const int32_t *d_members, int n_members, int max_nb_items, size_t lds,
                                   hipStream_t s);
hipError_t launch_edge_finish_multi(const EdgeArgs *d_args, int P, int max_nb_edge, hipStream_t s);

// ---- stage timing ------------------------------------------------------------
enum Stage { kStSample = 0, kStNearest, kStSteer, kStEdge, kStInsert, kStBridgeSel, kStBridgeEdge, kStPublish,
             kStEnd, kNumStages };
void prof_mark(st_problem *p, int stage, hipStream_t s);

// ---- nearest node and the extension pipeline --------------------------------
int nearest_set(st_problem *p, int32_t set, int32_t metric, int32_t sigma, int64_t M, const float *xq,
                int32_t *idx_out, float *dist_out, hipStream_t s);
// bucket (sample_batch): the sampler also buckets its workers by nearest-node
// set; bucketed (extend_batch): the samples were so bucketed (no separate
// bucketing kernel).  Both are set for the planner's own iterations.
int sample_batch(st_problem *p, int64_t iter, int64_t B, const st_samples &out, hipStream_t s, bool bucket);
int extend_batch(st_problem *p, int64_t B, const st_samples &in, const st_extend_out *out, hipStream_t s,
                 bool bucketed);
int work_reserve(st_problem *p, int64_t B);
void work_free(st_problem *p);
void graphs_free(st_problem *p);

// ---- allocation ------------------------------------------------------------
hipError_t launch_roots_update(st_problem *p, hipStream_t s);

}  // namespace st
