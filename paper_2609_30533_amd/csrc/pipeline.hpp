// pipeline.hpp -- launch records of the extend pipeline's kernels (one
// record per kernel and problem) and the many-problem launch description.
#pragma once

#include <vector>

#include "st_internal.hpp"

namespace st {

struct SampleArgs {
    SceneDev sc;
    WindowsDev win;
    const PlanDev *pl;
    int32_t variant, N;
    float p_guided, p_new;
    uint32_t seed, pid;
    int64_t iter, B;
    double t_min, t_max;  // arrival range (the learned histogram spans it)
    st_samples out;
    int32_t nb;           // blocks (many-problem launches)
    int32_t nw_lds;       // guided windows staged in LDS after the scene (0: read from device memory)
    // internal iterations: the sampler also buckets its workers by
    // nearest-node set, clears their keys and takes the batch's snapshot
    // (null bcnt: samples for a caller, no bucketing)
    int32_t n_pools;
    int32_t *bcnt, *border;
    unsigned long long *keys;
};

struct PrepArgs {
    PlanDev *pl;
    int32_t variant, n_pools, d;
    int64_t B;
    st_samples s;
    int32_t *bcnt, *border;  // nearest-node buckets (counters overwritten)
    unsigned long long *keys;
};

struct ScanArgs {
    TreeDev tree;
    const PlanDev *pl;
    int32_t use_snap, variant;
    float v;
    // query q: coordinate j at qx[q sq + j sj] (j < d), time at qt[q st]
    const float *qx, *qt;
    int64_t sq, sj, st;
    // queries per tile: bmode 0 from the tile list (identity query order);
    // 1 nearest-node buckets (sets = pools); 2 bridge buckets (two sets)
    int32_t bmode;
    const int4 *tiles;
    const int32_t *n_tiles;
    const int32_t *bcnt, *border;
    int64_t bstride;
    unsigned long long *keys;  // nearest node: per-query atomic minimum
    unsigned long long *pkey;  // bridges: [nch][pstride]
    int32_t *pidx;
    int64_t pstride;
    int32_t nch;
};

struct SteerArgs {
    SceneDev sc;
    TreeDev tree;
    const PlanDev *pl;
    int32_t variant;
    float eta;
    int64_t B;
    st_samples s;
    Work w;
};

struct InsertArgs {
    SceneDev sc;
    TreeDev tree;
    PlanDev *pl;
    int32_t variant;
    int64_t B;
    st_samples s;
    Work w;  // also: clears the nearest-node bucket counters, fills the bridge buckets
};

struct BridgeArgs {
    TreeDev tree;
    int64_t B;
    int32_t nch;
    const int8_t *dir;
    Work w;  // the bridge buckets give the advanced workers (one wave each, densely)
};

struct PublishArgs {
    PlanDev *pl;
    int64_t B;
    const int8_t *dir;
    Work w;
    st_extend_out out;
    // bridge edge results still in the edge buffers (finish step done here)
    EdgeBufs eb;
    unsigned long long *work_br;  // two work counters
};

struct RootsArgs {
    SceneDev sc;
    TreeDev tree;
    WindowsDev win;
    PlanDev *pl;
    int32_t variant, N;
    int32_t no_recycling;  // keep the initial roots (deactivation only)
};

// Every record of one iteration of one problem.
struct IterArgs {
    PrepArgs prep_nn;
    ScanArgs scan_nn, scan_br;
    SteerArgs steer;
    EdgeArgs edge_ext, edge_br;
    InsertArgs insert;
    BridgeArgs merge;
    PublishArgs publish;
    RootsArgs roots;
    int mt_nn, mt_br;  // query tiles at most
};

// bucket: the sampler of an internal iteration (buckets its workers; the
// extend step then runs without the separate bucketing kernel)
SampleArgs make_sample_args(const st_problem *p, int64_t iter, int64_t B, const st_samples &out, bool bucket);
// nch_*: node slices per scan tile; min_item_blocks: least blocks of the edge
// item kernel; launch_edges: edges of the whole launch (for the automatic
// lanes per state).
void make_iter_args(const st_problem *p, int64_t B, const st_samples &in, const st_extend_out *out, int nch_nn,
                    int nch_br, int min_item_blocks, int64_t launch_edges, IterArgs &a);

// Problems whose scene compiles to the same kernel instances (robot kind,
// obstacle tile, obstacle-time mode, lanes per state).
struct BatchClass {
    SceneDev key;           // kind, ot and obs_mode select the instance
    int split_ext, split_br;  // lanes per state (log2) of the two edge launches
    const int32_t *members; // device: record indices
    int n;                  // members
    int nb_sample, nb_items_ext, nb_items_br, nb_flat, nb_bcheck;  // grid maxima over the members
    size_t lds;             // dynamic LDS, maximum over the members
    size_t lds_sample;      // the sampler's (scene and guided windows), maximum over the members
};

// Samples per iteration of a batch member at most (a grid dimension).
constexpr int kBatchMaxSamples = 65535;

// Device arrays of records (P problems) and grid maxima for one iteration of
// every problem of a batch.
struct BatchLaunch {
    int P = 0;
    const SampleArgs *sample = nullptr;
    const ScanArgs *scan_nn = nullptr, *scan_br = nullptr;
    const SteerArgs *steer = nullptr;
    const EdgeArgs *edge_ext = nullptr, *edge_br = nullptr;
    const InsertArgs *insert = nullptr;
    const BridgeArgs *merge = nullptr;
    const PublishArgs *publish = nullptr;
    const RootsArgs *roots = nullptr;
    const int32_t *ir_members = nullptr, *rr_members = nullptr, *all_members = nullptr;
    int n_ir = 0, n_rr = 0;
    int mt_nn_ir = 0, mt_nn_rr = 0, mt_br = 0, nch = 1, nb_worker = 0, nb_edge = 0, max_pools = 0;
    int ins_threads = 64;  // insertion block size for the largest member
    int scan_tq = 256;     // queries per scan tile and scan block size (256 or 64)
    bool ext_flat = true;  // every member's extension edges take the flattened path
    std::vector<BatchClass> classes;
};

int launch_batch_iteration(const BatchLaunch &L, hipStream_t s);
int start_check(st_problem *p, bool *start_free, bool *trivial);
int fetch_path(st_problem *p, hipStream_t s, st_path *out);
st_samples work_samples_of(st_problem *p);
size_t scene_lds_bytes(const SceneDev &sc);
// Dynamic LDS of the sampler: the scene, then (interval root) the guided
// windows lo, hi, cum as doubles when they fit.
size_t sample_lds_bytes(const st_problem *p, int32_t *nw_lds);
int nch_for_tiles(int tiles);
int max_query_tiles(int64_t B, int n_sets);

}  // namespace st
