// extend.hip -- the batched space-time extend step (Alg. 1) driven by the
// interval-root (Alg. 2) or root-recycling (Alg. 3) allocation.
//
// One batch is a fixed sequence of kernels on one stream:
//   sample   a1  Philox draws -> direction, group/slot, root time T, root check,
//                q_r, t_r (Eq. 6), p_new rule
//   prep         snapshot of pool counts and U; workers bucketed by node set
//   scan     a2  nearest node: tiles of 64 queries (one per lane) stream a
//                node set from HBM through LDS; packed (distance, index) keys
//                are merged with 64-bit atomicMin, so ties go to the lowest index
//   steer    a3  alpha = min(1, eta/rho) (interval root) or Eq. 8 (recycling)
//   check    a4  edge checks (collide.hip), any-hit early exit
//   insert   a5  one block per pool: prefix sum over workers in order, slots
//                after the snapshot count, virtual roots materialised first
//   bridge   a6  best-ranked candidate in the opposite set (arrival, rho, index),
//                per-chunk partials merged per worker, then its edge check
//   publish  a7  lexicographic minimum of (U', C', worker) against (U, C)
//   roots    a8/a9 allocation update after a strict drop of U
// Every worker sees the trees as they were when the batch started.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "edge_flat.hpp"
#include "pipeline.hpp"
#include "rng.hpp"
#include "st_internal.hpp"

namespace st {

constexpr int kTileQ = 256;  // queries per scan tile (one per thread)
constexpr int kMaxNch = 256;  // node slices per scan tile at most
constexpr unsigned long long kNoKey = ~0ull;
constexpr int kSetAllBackward = -2;

__device__ __forceinline__ unsigned long long pack_key(float dist_key, int32_t idx) {
    return ((unsigned long long)__float_as_uint(dist_key) << 32) | (uint32_t)idx;
}

__device__ __forceinline__ int worker_pool(int8_t dir, int32_t grp) { return dir == 0 ? 0 : 1 + grp; }

// ---------------------------------------------------------------------------
// a1: sampling
// ---------------------------------------------------------------------------


// Root time for group g of the current interval-root allocation, in double:
// with probability p_guided (when the guided windows below Ubar are not empty)
// a portion of the group's guided share chosen in proportion to its length and
// a uniform time inside it; otherwise uniform on I_g.
// The windows' lo, hi and cum arrays are read from wlo, whi, wcum (LDS when
// the sampler staged them, else the device copies in w).
__device__ double ir_root_time(const WindowsDev &w, const double *wlo, const double *whi, const double *wcum,
                               double Ubar, double G, int jstar, int g, const uint32_t *u, float p_guided) {
    const double L = w.L;
    const int N = w.N;
    if (unit24f(u[1]) < p_guided && G > 0.0 && jstar > 0) {
        const double c_lo = G * g / N, c_hi = G * (g + 1) / N;
        const double c = c_lo + unit24d(u[2]) * (c_hi - c_lo);
        // window j with cum[j] <= c < cum[j] + len_j
        int lo = 0, hi = jstar - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (wcum[mid] <= c) lo = mid;
            else hi = mid - 1;
        }
        const int j = lo;
        const double len = fmin(whi[j], Ubar) - wlo[j];
        const double a = fmax(c_lo, wcum[j]), b = fmin(c_hi, wcum[j] + len);
        return wlo[j] + (a - wcum[j]) + unit24d(u[3]) * (b - a);
    }
    const double width = (Ubar - L) / N;
    const double I0 = L + g * width, I1 = L + (g + 1) * width;
    return I0 + unit24d(u[3]) * (I1 - I0);
}

// Adds `amount` lanes' worth to bucket[set] with one atomic per distinct set
// in the wave; returns each lane's position among the lanes of its set (in
// lane order) plus the bucket's previous value.  Every lane must call it.
__device__ __forceinline__ int wave_bucket_add(int *bucket, int set) {
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(set >= 0);
    int pos = -1;
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int ls = __shfl(set, leader, 64);
        const uint64_t same = __ballot(set == ls) & pending;
        int base = 0;
        if (lane == leader) base = atomicAdd(&bucket[ls], __popcll(same));
        base = __shfl(base, leader, 64);
        if (set == ls) pos = base + __popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    return pos;
}

// MULTI: many problems per launch; blockIdx.y picks the problem's record
// (through the member list of its scene class) and blocks past the problem's
// own grid leave at once.  The kernels below follow this convention, except
// the scans (member in blockIdx.z) and the bridge check (member in
// blockIdx.x, so that members vary fastest).
// Lanes per worker in the sampler: the arm's root check (q_g, T) shares the
// spheres out among four lanes; every lane of a worker draws the same numbers.
template <int KIND>
constexpr int sample_lanes() { return KIND == kTranslate ? 1 : 4; }

template <int KIND, int OT, int OBS, bool MULTI>
__global__ __launch_bounds__(256) void k_sample(SampleArgs a0, const SampleArgs *__restrict__ av,
                                                const int32_t *__restrict__ members) {
    extern __shared__ float4 lds[];
    const SampleArgs &a = MULTI ? av[members[blockIdx.y]] : a0;
    if (MULTI && (int)blockIdx.x >= a.nb) return;
    const SceneDev &sc = a.sc;
    const bool ir = a.variant == ST_INTERVAL_ROOT;
    // the plan state the sampler reads, loaded ahead of the staging barrier
    // so that its latency overlaps the staging (a negative iteration means
    // "the planner's own counter", as in graph replays)
    const PlanDev *pl = a.pl;
    const int64_t iter = a.iter >= 0 ? a.iter : (int64_t)pl->iter;
    const float prop_mix = pl->prop_mix, U_now = pl->U;
    const int32_t done = pl->done, n_active = pl->n_active, jstar = pl->jstar;
    const double Ubar = pl->Ubar, Gsum = pl->G;
    const bool snap_block = a.bcnt && blockIdx.x == 0;
    const int32_t snap_count = snap_block && (int)threadIdx.x < a.n_pools ? pl->count[threadIdx.x] : 0;
    // interval root: the guided windows go to LDS behind the scene, so the
    // binary search of a root time reads LDS, not device memory
    const int nwl = ir ? a.nw_lds : 0;
    double *wl = reinterpret_cast<double *>(lds + sc.lds_f4);
    for (int i = threadIdx.x; i < nwl; i += blockDim.x) {
        const double x0 = a.win.lo[i], x1 = a.win.hi[i], x2 = a.win.cum[i];
        wl[i] = x0;
        wl[nwl + i] = x1;
        wl[2 * nwl + i] = x2;
    }
    if (ir) stage_obstacles(sc, lds);
    constexpr int SL = sample_lanes<KIND>();
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = gt / SL;
    const int part = (int)(gt % SL);
    const bool act = w < a.B;
    uint32_t u[28];
    const bool learned = prop_mix > 0.f;
    const int nblk = learned ? 7 : 4;
#pragma unroll
    for (int b = 0; b < 7; ++b) {
        if (b >= nblk) break;
        const U4 r = philox4x32_10((uint32_t)iter, (uint32_t)w, (uint32_t)b, 0u, a.seed, a.pid);
#pragma unroll
        for (int k = 0; k < 4; ++k) u[4 * b + k] = r.x[k];
    }
    const int8_t dir = (int8_t)((w + iter) & 1);
    uint8_t flags = 0;
    int32_t g = 0;
    float T = 0.f, tr = 0.f;
    float q[kMaxDof];
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j)
        q[j] = j < sc.d ? sc.q_lo[j] + unit24f(u[4 + j]) * (sc.q_hi[j] - sc.q_lo[j]) : 0.f;
    bool check_root = false;
    // learned draw: (q, t) from the mixture, T from the arrival histogram
    const bool use_net = learned && unit24f(u[13]) < prop_mix;
    float y7 = 0.f;
    if (use_net) {
        flags |= ST_FLAG_LEARNED;
        int c = 0;
        while (c < 7 && !(unit24f(u[14]) < pl->prop_wcum[c])) ++c;
        float nrm[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // Box-Muller (Box and Muller, 1958) from two uniforms in (0, 1] and [0, 1)
            const float r = sqrtf(-2.f * __logf(1.f - unit24f(u[16 + 2 * k])));
            float sn, cs;
            __sincosf(6.28318530717958648f * unit24f(u[17 + 2 * k]), &sn, &cs);
            nrm[2 * k] = r * cs;
            nrm[2 * k + 1] = r * sn;
        }
        bool inside = true;
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) {
            if (j < sc.d) {
                q[j] = 3.14159265358979324f * fmaf(pl->prop_sd[c * 8 + j], nrm[j], pl->prop_mu[c * 8 + j]);
                inside = inside && q[j] >= sc.q_lo[j] && q[j] <= sc.q_hi[j];
            }
        }
        y7 = 60.f * fmaf(pl->prop_sd[c * 8 + 7], nrm[7], pl->prop_mu[c * 8 + 7]);
        if (!inside) flags |= ST_FLAG_SKIP;
    }
    if (ir) {
        g = index24(u[0], a.N);
        if (!act || done) {
            flags |= ST_FLAG_SKIP;
        } else if (use_net) {
            int b = 0;
            while (b < 31 && !(unit24f(u[15]) < pl->prop_hcum[b])) ++b;
            const double w = (a.t_max - a.t_min) / 32.0;
            const double Td = a.t_min + ((double)b + unit24d(u[24])) * w;
            const double L = a.win.L;
            if (!(Td >= L && Td < Ubar)) {
                flags |= ST_FLAG_SKIP;
            } else {
                // the group whose uniform interval holds T
                const int gi = (int)floor((Td - L) / ((Ubar - L) / a.N));
                g = gi < 0 ? 0 : (gi >= a.N ? a.N - 1 : gi);
                T = (float)Td;
                check_root = !(flags & ST_FLAG_SKIP);
            }
        } else {
            T = nwl > 0 ? (float)ir_root_time(a.win, wl, wl + nwl, wl + 2 * nwl, Ubar, Gsum, jstar, g, u, a.p_guided)
                        : (float)ir_root_time(a.win, a.win.lo, a.win.hi, a.win.cum, Ubar, Gsum, jstar, g, u,
                                              a.p_guided);
            check_root = true;
        }
    } else if (act && dir == 1) {
        const int64_t k = w >> 1;
        const int na = n_active;
        if (na == 0) {
            flags |= ST_FLAG_SKIP;
        } else {
            g = pl->active_list[k % na];
            T = pl->slotT[g];
        }
    }
    if (ir) {
        // the group's earliest root, loaded ahead of the root check's arithmetic
        const float min_root = check_root && dir == 1 ? pl->minRootT[g] : 0.f;
        // the proposed root (q_g, T) is checked at its own time
        const bool hit = goal_hits<OT, OBS, SL>(sc, lds, T, check_root, part);
        if (check_root) {
            if (hit) flags |= ST_FLAG_SKIP;
            // Eq. 6: t_r ~ U[D(q_s, q_r)/v, T - D(q_r, q_g)/v], empty interval rejected
            float ds = 0.f, dg = 0.f;
#pragma unroll
            for (int j = 0; j < kMaxDof; ++j) {
                if (j < sc.d) {
                    const float e1 = q[j] - sc.q_s[j], e2 = sc.q_g[j] - q[j];
                    ds = fmaf(e1, e1, ds);
                    dg = fmaf(e2, e2, dg);
                }
            }
            const float lo = sqrtf(ds) / sc.v, hi = T - sqrtf(dg) / sc.v;
            if (hi < lo) flags |= ST_FLAG_SKIP;
            else if (use_net) {
                // the learned time must satisfy the same bounds
                tr = y7;
                if (!(tr >= lo && tr <= hi)) flags |= ST_FLAG_SKIP;
            } else {
                tr = lo + unit24f(u[11]) * (hi - lo);
            }
            if (dir == 1 && (!(min_root < U_now) || unit24f(u[12]) <= a.p_new)) flags |= ST_FLAG_USE_NEW;
        }
    }
    if (a.bcnt) {
        // the worker's nearest-node set (the forward tree, or its backward
        // group or slot; a new interval root has none: its root is the node),
        // its place in that set's bucket, its empty key, and the snapshot
        // every worker of this batch sees (counts and U before any insert)
        // (places within the block from LDS counters, then one global atomic
        // per set and block)
        __shared__ int s_bcnt[kMaxPools], s_bbase[kMaxPools];
        if ((int)threadIdx.x < a.n_pools) s_bcnt[threadIdx.x] = 0;
        __syncthreads();
        int set = -1;
        if (act && part == 0 && !(flags & ST_FLAG_SKIP)) {
            if (dir == 0) set = 0;
            else if (g >= 0 && g < a.n_pools - 1 && !(ir && (flags & ST_FLAG_USE_NEW))) set = 1 + g;
        }
        const int pos = wave_bucket_add(s_bcnt, set);
        __syncthreads();
        if ((int)threadIdx.x < a.n_pools && s_bcnt[threadIdx.x] > 0)
            s_bbase[threadIdx.x] = atomicAdd(&a.bcnt[threadIdx.x], s_bcnt[threadIdx.x]);
        __syncthreads();
        if (set >= 0) a.border[(int64_t)set * a.B + s_bbase[set] + pos] = (int32_t)w;
        if (act && part == 0) a.keys[w] = kNoKey;
        if (snap_block) {
            PlanDev *plw = const_cast<PlanDev *>(pl);
            const int tid = threadIdx.x;
            if (tid < a.n_pools) plw->count_snap[tid] = snap_count;
            if (tid == 0) {
                plw->U_snap = U_now;
                plw->improved = 0;
            }
        }
    }
    if (!act || part != 0) return;
    a.out.dir[w] = dir;
    a.out.flags[w] = flags;
    a.out.grp[w] = g;
    a.out.T[w] = T;
    for (int j = 0; j < sc.d; ++j) a.out.qr[(int64_t)j * a.B + w] = q[j];
    a.out.tr[w] = tr;
}

// ---------------------------------------------------------------------------
// bucketing of queries by node set
// ---------------------------------------------------------------------------


// Bucketing of caller-given samples (st_extend_batch; an internal iteration's
// sampler does this itself): each worker's nearest-node set, its place in the
// set's bucket, its empty key, and the snapshot of the batch.  One block; the
// counters are overwritten.
__global__ __launch_bounds__(1024) void k_prep(PrepArgs a) {
    __shared__ int cnt[kMaxPools];
    const int tid = threadIdx.x;
    for (int i = tid; i < a.n_pools; i += blockDim.x) cnt[i] = 0;
    // the snapshot every worker of this batch sees (one pool per thread),
    // loaded here and stored after the worker loads
    int32_t snap_count = 0;
    float snap_U = 0.f;
    if (tid < a.n_pools) snap_count = a.pl->count[tid];
    if (tid == 0) snap_U = a.pl->U;
    __syncthreads();
    // R consecutive workers per thread and pass, all loads before the stores
    constexpr int R = 4;
    for (int64_t base = 0; base < a.B; base += (int64_t)blockDim.x * R) {
        uint8_t f[R];
        int8_t dr[R];
        int32_t g[R];
        // unconditional loads (a worker past B reads worker B - 1 and is
        // ignored): guarded loads would each wait before the next one issues
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t w = base + (int64_t)tid * R + r;
            const int64_t wc = w < a.B ? w : a.B - 1;
            f[r] = a.s.flags[wc];
            dr[r] = a.s.dir[wc];
            g[r] = a.s.grp[wc];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t w = base + (int64_t)tid * R + r;
            int set = -1;
            if (w < a.B && !(f[r] & ST_FLAG_SKIP)) {
                if (dr[r] == 0) set = 0;
                else if (g[r] >= 0 && g[r] < a.n_pools - 1 &&
                         !(a.variant == ST_INTERVAL_ROOT && (f[r] & ST_FLAG_USE_NEW)))
                    set = 1 + g[r];
            }
            if (w < a.B) a.keys[w] = kNoKey;
            const int pos = wave_bucket_add(cnt, set);
            if (set >= 0) a.border[(int64_t)set * a.B + pos] = (int32_t)w;
        }
    }
    if (tid < a.n_pools) a.pl->count_snap[tid] = snap_count;
    if (tid == 0) {
        a.pl->U_snap = snap_U;
        a.pl->improved = 0;
    }
    __syncthreads();
    if (tid < a.n_pools) a.bcnt[tid] = cnt[tid];
}

// ---------------------------------------------------------------------------
// a2 / a6: node-set scans
// ---------------------------------------------------------------------------

enum { kScanRho = 0, kScanConfig = 1, kScanBridge = 2 };
constexpr int kMinSliceNodes = 64;  // nearest-node scans: nodes per slice at least


// One block = one tile of up to TQ queries (one per thread) against the
// y-th of nch slices of its node set.  The set is a single pool or the
// concatenation of the backward pools; nodes stream through LDS in rounds of
// TQ (each thread loads one node, coalesced per SoA row), and the next round
// is fetched into registers while the current one is scanned.  TQ is 256, or
// 64 for a batch of problems with at most 64 samples each: their tiles hold a
// few queries, and one-wave blocks keep four times as many of the launch's
// (mostly empty) blocks in flight.
template <int MODE, bool MULTI, int TQ = kTileQ>
__global__ __launch_bounds__(TQ) void k_scan(ScanArgs a0, const ScanArgs *__restrict__ av,
                                             const int32_t *__restrict__ members) {
    __shared__ __align__(16) float sx[TQ][8];
    __shared__ float sT[TQ];
    __shared__ int32_t sI[TQ];
    __shared__ int32_t s_pool[kMaxPools + 1], s_pre[kMaxPools + 1], s_cnt[kMaxPools + 1];
    __shared__ int32_t s_np;
    const ScanArgs &a = MULTI ? av[members[blockIdx.z]] : a0;
    if (MULTI && (int)blockIdx.y >= a.nch) return;
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const PlanDev *pl = a.pl;
    const float U = a.use_snap ? pl->U_snap : pl->U;  // loaded ahead of the set-up barriers
    int4 tile;             // set, first query, queries, sigma
    int64_t qrow = -1;     // bucket row of the tile's queries (-1: identity order)
    int64_t prow = -1;     // bridge buckets: the tile's first query in the two buckets' order
    if (a.bmode == 0) {
        if (t >= a.n_tiles[0]) return;
        tile = a.tiles[t];
    } else {
        // tile t is tile kt of bucket sb: the buckets' tiles in set order,
        // from the counts (read together, then walked from LDS by every thread)
        __shared__ int32_t s_bc[kMaxPools];
        const int nsets = a.bmode == 1 ? a.tree.n_pools : 2;
        // (a block of 64 threads may have fewer threads than sets)
        for (int i = tid; i < nsets; i += TQ) s_bc[i] = a.bcnt[i];
        __syncthreads();
        int acc = 0, sb = 0, kt = -1;
        for (; sb < nsets; ++sb) {
            const int nt = (s_bc[sb] + TQ - 1) / TQ;
            if (t < acc + nt) {
                kt = t - acc;
                break;
            }
            acc += nt;
        }
        if (kt < 0) return;  // past the last tile (the same for the whole block)
        int set_id, sg;
        if (a.bmode == 1) {
            set_id = sb;
            sg = sb == 0 ? 1 : -1;
        } else {
            // a bridge from x_new in direction sigma needs sigma (t_y - t_new) > 0,
            // i.e. the nearest-node rule with the opposite sign: forward new
            // nodes into the backward forest, backward new nodes into the tree
            set_id = sb == 0 ? kSetAllBackward : 0;
            sg = sb == 0 ? -1 : 1;
        }
        tile = make_int4(set_id, kt * TQ, min(TQ, s_bc[sb] - kt * TQ), sg);
        qrow = (int64_t)sb * a.bstride;
        if (a.bmode == 2) prow = (sb == 0 ? 0 : (int64_t)s_bc[0]) + (int64_t)kt * TQ;
    }
    const int set = tile.x, n = tile.z;
    const float sv = (float)tile.w * a.v;  // sigma * v
    const int d = a.tree.d;
    // pools of the set and their prefix sums: the counts are loaded by one
    // thread per pool, the prefix is formed from LDS
    const int p_lo = set >= 0 ? set : 1, p_hi = set >= 0 ? set + 1 : a.tree.n_pools;
    for (int p = p_lo + tid; p < p_hi; p += blockDim.x) {
        int c = a.use_snap ? pl->count_snap[p] : pl->count[p];
        if (a.variant == ST_ROOT_RECYCLING && set < 0 && !pl->slot_active[p - 1]) c = 0;
        s_cnt[p - p_lo] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int k = 0, acc = 0;
        for (int p = p_lo; p < p_hi; ++p) {
            const int c = s_cnt[p - p_lo];
            if (c <= 0) continue;
            s_pool[k] = p;
            s_pre[k] = acc;
            acc += c;
            ++k;
        }
        s_pre[k] = acc;
        s_np = k;
    }
    __syncthreads();
    const int np = s_np;
    const int64_t total = s_pre[np];
    // nearest-node scans of small node sets use fewer slices (each of at least
    // kMinSliceNodes nodes); the blocks past them leave (the keys they would
    // merge into start empty).  Bridge scans keep every slice: their merge
    // reads one partial result per slice.
    int nch = a.nch;
    if (MODE != kScanBridge) {
        const int64_t want = (total + kMinSliceNodes - 1) / kMinSliceNodes;
        nch = (int)min<int64_t>(nch, max<int64_t>(want, 1));
        if ((int)blockIdx.y >= nch) return;
    }
    // lanes per query: as many as the tile's queries leave free (a power of
    // two, at most a wave); lane `sub` of a query takes every L-th node of a
    // round, and the query's L lanes combine their bests at the end
    int lq_shift = 0;
    while (lq_shift < 6 && n * (2 << lq_shift) <= TQ) ++lq_shift;
    const int L = 1 << lq_shift, qs = tid >> lq_shift, sub = tid & (L - 1);
    const bool act = qs < n;
    const int q = act ? (qrow >= 0 ? a.border[qrow + tile.y + qs] : tile.y + qs) : 0;
    const int64_t c0 = (int64_t)blockIdx.y * total / nch, c1 = (int64_t)(blockIdx.y + 1) * total / nch;
    float qx[kMaxDof];
    float aq = 0.f;
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j) qx[j] = (act && j < d) ? a.qx[(int64_t)q * a.sq + (int64_t)j * a.sj] : 0.f;
    if (act) aq = sv * a.qt[(int64_t)q * a.st];
    float best = INFINITY, bestT = INFINITY;
    int32_t bi = -1;
    const float *X = a.tree.x;
    const int64_t total_cap = a.tree.total;
    const float nanf_ = __int_as_float(0x7fc00000);
    // register stage for one node
    float rx[8];
    float rT = 0.f;
    int32_t rI = -1;
    auto fetch = [&](int64_t vbase) {
        const int64_t v = vbase + tid;
        rI = -1;
        if (v < c1) {
            int k = 0;
            while (k + 1 < np && v >= s_pre[k + 1]) ++k;
            const int p = s_pool[k];
            const int64_t gi = pool_base(a.tree, p) + (v - s_pre[k]);
            // slots past d hold 0 (as the query's do): they add exact zeros
#pragma unroll
            for (int j = 0; j < kMaxDof; ++j) rx[j] = j < d ? X[(int64_t)j * total_cap + gi] : 0.f;
            float tn = X[(int64_t)d * total_cap + gi];
            const bool filt = a.variant == ST_INTERVAL_ROOT && p > 0;
            rT = (filt || MODE == kScanBridge) ? a.tree.rootT[gi] : 0.f;
            // inactive backward trees (root at or after U) are hidden behind a NaN time
            if (filt && !(rT < U)) tn = nanf_;
            rx[7] = sv * tn;
            rI = (int32_t)gi;
        }
    };
    if (c0 < c1) fetch(c0);
    for (int64_t c = c0; c < c1; c += TQ) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j) sx[tid][j] = rx[j];
        sT[tid] = rT;
        sI[tid] = rI;
        __syncthreads();
        if (c + TQ < c1) fetch(c + TQ);
        const int m = (int)min<int64_t>(TQ, c1 - c);
        if (act) {
            // a node is two 16-byte broadcast reads (all eight slots, the
            // unused ones ignored); unrolled so that the reads of several
            // nodes are in flight together.  The round's best node is kept
            // as its LDS slot and its index read once after the round.
            const float4 *sx4 = reinterpret_cast<const float4 *>(&sx[0][0]);
            int kb = -1;
#pragma unroll 8
            for (int k = sub; k < m; k += L) {
                const float4 lo = sx4[2 * k], hi = sx4[2 * k + 1];
                const float xs[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
                // every slot: those past d are 0 on both sides and add exact zeros
                float D2 = 0.f;
#pragma unroll
                for (int j = 0; j < kMaxDof; ++j) {
                    const float e = xs[j] - qx[j];
                    D2 = fmaf(e, e, D2);
                }
                if (MODE == kScanConfig) {
                    if (D2 < best) { best = D2; kb = k; }
                } else {
                    // Eq. 7: admissible iff sigma (t_q - t) > 0 and D <= v sigma (t_q - t)
                    const float vd = aq - xs[7];
                    const float w2 = vd * fabsf(vd);
                    const bool adm = (D2 <= w2) && (w2 > 0.f);
                    const float key = D2 + w2;
                    if (MODE == kScanRho) {
                        if (adm && key < best) { best = key; kb = k; }
                    } else {
                        const float arr = set < 0 ? sT[k] : 0.f;
                        if (adm && (arr < bestT || (arr == bestT && key < best))) {
                            bestT = arr;
                            best = key;
                            kb = k;
                        }
                    }
                }
            }
            if (kb >= 0) bi = sI[kb];
        }
    }
    // the query's lanes combine (every lane of the wave takes part): the
    // least key, ties to the least node index, as one lane walking all the
    // nodes in order would keep
    if (MODE == kScanBridge) {
        unsigned long long pk =
            bi < 0 ? kNoKey : (((unsigned long long)__float_as_uint(bestT) << 32) | __float_as_uint(best));
        uint32_t pi = (uint32_t)bi;
        for (int o = 1; o < L; o <<= 1) {
            const unsigned long long ok = __shfl_xor(pk, o, 64);
            const uint32_t oi = __shfl_xor(pi, o, 64);
            if (ok < pk || (ok == pk && oi < pi)) {
                pk = ok;
                pi = oi;
            }
        }
        if (!act || sub != 0) return;
        // a bridge query's row: its place in the two buckets (the bridge
        // check's wave index, known there before the worker is), else the query
        const int64_t r = prow >= 0 ? prow + qs : q;
        a.pkey[r * a.pstride + blockIdx.y] = pk;
        a.pidx[r * a.pstride + blockIdx.y] = (int32_t)pi;
    } else {
        unsigned long long key = bi >= 0 ? pack_key(best, bi) : kNoKey;
        for (int o = 1; o < L; o <<= 1) {
            const unsigned long long ok = __shfl_xor(key, o, 64);
            key = ok < key ? ok : key;
        }
        if (!act || sub != 0 || key == kNoKey) return;
        atomicMin(&a.keys[q], key);
    }
}

// ---------------------------------------------------------------------------
// a3: steering
// ---------------------------------------------------------------------------


// Steering of worker w (all its loads first, its records written last):
// the nearest node x_n from the scan's key, or the virtual root (q_g, T);
// x_new; the [0, H] check.  Writes the worker's status (TRAPPED / SKIPPED
// until the insert decides), new index (-1), edge flag, parent and, when the
// extension is to be checked, x_n, x_new, the cost and root time of x_new.
// Returns whether the extension edge (x_n, x_new) is to be checked, with both
// endpoints in xn / xnew.
__device__ __forceinline__ bool steer_worker(const SteerArgs &a, int64_t w, float (&xn)[kMaxDof + 1],
                                             float (&xnew)[kMaxDof + 1]) {
    const SceneDev &sc = a.sc;
    const int d = sc.d, W = d + 1;
    const Work &k = a.w;
    // every load is issued before the first store (a store ahead of a load
    // would make the load's wait include the store's completion)
    const uint8_t f = a.s.flags[w];
    const int8_t dir = a.s.dir[w];
    const int32_t g = a.s.grp[w];
    const unsigned long long key = k.nn_key[w];
    const float Tw = a.s.T[w];
    float xr[kMaxDof + 1];
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j) xr[j] = j < d ? a.s.qr[(int64_t)j * a.B + w] : 0.f;
    xr[d] = a.s.tr[w];
    // a backward worker must name an existing group / slot
    const bool skip = (f & ST_FLAG_SKIP) || (dir != 0 && (g < 0 || g >= a.tree.n_pools - 1));
    const bool virt = a.variant == ST_INTERVAL_ROOT && dir == 1 && (f & ST_FLAG_USE_NEW);
    int8_t status = skip ? ST_STATUS_SKIPPED : ST_STATUS_TRAPPED;
    bool ok = !skip && (virt || key != kNoKey);  // TRAPPED when nothing is admissible
    int32_t idx = -1;
    float cost0 = 0.f, root0 = 0.f;
    if (ok && virt) {
        for (int j = 0; j < d; ++j) xn[j] = sc.q_g[j];
        xn[d] = Tw;
        root0 = Tw;
    } else if (ok) {
        idx = (int32_t)(key & 0xffffffffu);
        for (int j = 0; j <= d; ++j) xn[j] = a.tree.x[(int64_t)j * a.tree.total + idx];
        cost0 = a.tree.cost[idx];
        root0 = dir == 0 ? 0.f : a.tree.rootT[idx];
    }
    float step = 0.f;
    if (ok) {
        const float sigma = dir == 0 ? 1.f : -1.f;
        float D2 = 0.f;
        for (int j = 0; j < d; ++j) {
            const float e = xr[j] - xn[j];
            D2 = fmaf(e, e, D2);
        }
        if (a.variant == ST_INTERVAL_ROOT) {
            const float vd = sigma * sc.v * (xr[d] - xn[d]);
            const float w2 = vd * fabsf(vd);
            if (!(D2 <= w2 && w2 > 0.f)) {
                ok = false;  // rho infinite
            } else {
                const float rho = sqrtf(0.5f * (D2 + w2));
                const float alpha = fminf(1.f, a.eta / rho);  // Alg. 1: same fraction in q and t
                for (int j = 0; j <= d; ++j) xnew[j] = fmaf(alpha, xr[j] - xn[j], xn[j]);
                float s2 = 0.f;
                for (int j = 0; j < d; ++j) {
                    const float e = xnew[j] - xn[j];
                    s2 = fmaf(e, e, s2);
                }
                step = sqrtf(s2);
            }
        } else {
            const float D = sqrtf(D2);
            if (!(D > 0.f)) {
                ok = false;  // no proposal
            } else {
                const float fr = fminf(1.f, a.eta / D);
                float s2 = 0.f;
                for (int j = 0; j < d; ++j) {
                    xnew[j] = fmaf(fr, xr[j] - xn[j], xn[j]);
                    const float e = xnew[j] - xn[j];
                    s2 = fmaf(e, e, s2);
                }
                step = sqrtf(s2);
                xnew[d] = xn[d] + sigma * step / sc.v;  // Eq. 8: maximum-speed timing
            }
        }
        if (ok && !(xnew[d] >= 0.f && xnew[d] <= sc.H)) ok = false;  // leaves [0, H]
    }
    k.status[w] = status;
    k.new_idx[w] = -1;
    k.edge_valid[w] = ok ? 1 : 0;
    k.parent[w] = ok ? idx : -1;
    if (!ok) return false;
    for (int j = 0; j <= d; ++j) {
        k.xn[w * W + j] = xn[j];
        k.xnew[w * W + j] = xnew[j];
    }
    k.cost_new[w] = cost0 + step;
    k.rootT_new[w] = root0;
    return true;
}

template <bool MULTI>
__global__ __launch_bounds__(256) void k_steer(SteerArgs a0, const SteerArgs *__restrict__ av) {
    const SteerArgs &a = MULTI ? av[blockIdx.y] : a0;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.B) return;
    float xn[kMaxDof + 1], xnew[kMaxDof + 1];
    (void)steer_worker(a, w, xn, xnew);
}

// Steering and the extension edge check in one launch (flattened path of
// short edges): each block steers its edges' workers itself (a3) and checks
// the resulting edges (a4), with no round trip through a separate launch.
template <int KIND, int OT, int OBS>
__device__ __forceinline__ void steer_flat_body(const SteerArgs &sa, const EdgeArgs &ea, float4 *lds, int bx) {
    const int d = sa.sc.d;
    edge_flat_body<KIND, OT, OBS>(ea, lds, bx, [&](int64_t e, float (&A)[kMaxDof + 1], float (&B)[kMaxDof + 1]) {
        float xn[kMaxDof + 1], xnew[kMaxDof + 1];
        if (!steer_worker(sa, e, xn, xnew)) return false;
        // both endpoints, earlier time first
        const bool sw = xn[d] > xnew[d];
#pragma unroll
        for (int j = 0; j <= kMaxDof; ++j) {
            A[j] = j <= d ? (sw ? xnew[j] : xn[j]) : 0.f;
            B[j] = j <= d ? (sw ? xn[j] : xnew[j]) : 0.f;
        }
        return true;
    });
}

template <int KIND, int OT, int OBS>
__global__ __launch_bounds__(64 * kFlatWaves) void k_steer_flat(SteerArgs sa, EdgeArgs ea) {
    extern __shared__ float4 lds[];
    steer_flat_body<KIND, OT, OBS>(sa, ea, lds, blockIdx.x);
}

template <int KIND, int OT, int OBS>
__global__ __launch_bounds__(64 * kFlatWaves) void k_steer_flat_multi(const SteerArgs *__restrict__ sv,
                                                                     const EdgeArgs *__restrict__ ev,
                                                                     const int32_t *__restrict__ members) {
    extern __shared__ float4 lds[];
    const int m = members[blockIdx.y];
    const EdgeArgs &ea = ev[m];
    if ((int64_t)blockIdx.x * kFlatGroups * ea.flat >= ea.E) return;
    steer_flat_body<KIND, OT, OBS>(sv[m], ea, lds, blockIdx.x);
}

// ---------------------------------------------------------------------------
// a5: insertion, one block per pool, workers in index order
// ---------------------------------------------------------------------------


template <bool MULTI>
__global__ __launch_bounds__(1024) void k_insert(InsertArgs a0, const InsertArgs *__restrict__ av) {
    __shared__ int wsum[32];
    __shared__ int s_total, s_last;
    __shared__ int s_bcnt[2], s_bbase[2];  // bridge bucket places of this pass
    const InsertArgs &a = MULTI ? av[blockIdx.y] : a0;
    const int p = blockIdx.x;
    if (MULTI && p >= a.tree.n_pools) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nw = blockDim.x >> 6;
    PlanDev *pl = a.pl;
    const Work &k = a.w;
    const int d = a.tree.d, W = d + 1;
    const int64_t base = pool_base(a.tree, p);
    const int64_t snap = pl->count_snap[p];
    const int64_t avail = pool_cap(a.tree, p) - snap;
    int64_t running = 0;
    if (tid == 0) s_last = 0;
    if (tid < 2) s_bcnt[tid] = 0;
    // the nearest-node buckets are consumed: empty for the next batch
    if (p == 0)
        for (int i = tid; i < a.tree.n_pools; i += blockDim.x) k.bcnt[i] = 0;
    // R consecutive workers per thread and pass; all their loads are issued
    // before any store
    constexpr int R = 4;
    for (int64_t c0 = 0; c0 < a.B; c0 += (int64_t)blockDim.x * R) {
        int need[R];
        int32_t par0[R];
        uint8_t ev[R], ef[R];
        int8_t dr[R];
        int32_t gr[R];
        // unconditional loads (a worker past B reads worker B - 1 and is
        // ignored): guarded loads would each wait before the next one issues
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t w = c0 + (int64_t)tid * R + r;
            const bool in = w < a.B;
            const int64_t wc = in ? w : a.B - 1;
            const uint8_t v0 = k.edge_valid[wc], f0 = k.edge_free[wc];
            const int8_t d0 = a.s.dir[wc];
            const int32_t g0 = a.s.grp[wc], p0 = k.parent[wc];
            ev[r] = in ? v0 : 0;
            ef[r] = in ? f0 : 0;
            dr[r] = in ? d0 : 0;
            gr[r] = in ? g0 : 0;
            par0[r] = in ? p0 : 0;
        }
        int tot = 0;
        bool trapped[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            need[r] = 0;
            trapped[r] = false;
            if (ev[r] && worker_pool(dr[r], gr[r]) == p) {
                if (!ef[r]) trapped[r] = true;  // the extension collides
                else need[r] = par0[r] < 0 ? 2 : 1;
            }
            tot += need[r];
        }
        // the payload of this pool's new nodes, every load in flight together
        // and ahead of the first store (a load behind a store waits for it)
        // (no default values: a select on a guarded load would wait for it)
        float xv[R][kMaxDof + 1], cn[R], rn[R], Tw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t w = c0 + (int64_t)tid * R + r;
            if (need[r] > 0) {
#pragma unroll
                for (int jj = 0; jj <= kMaxDof; ++jj)
                    if (jj <= d) xv[r][jj] = k.xnew[w * W + jj];
                cn[r] = k.cost_new[w];
                rn[r] = k.rootT_new[w];
                Tw[r] = a.s.T[w];
            }
        }

        // block-wide exclusive prefix of the threads' totals (worker order)
        int incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int i = 0; i < nw; ++i) {
                const int v = wsum[i];
                wsum[i] = acc;
                acc += v;
            }
            s_total = acc;
        }
        __syncthreads();
        int64_t off = running + wsum[wv] + incl - tot;
        int bset[R];  // bridge bucket of an inserted worker (0 forward, 1 backward)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            bset[r] = -1;
            if (need[r] == 0) continue;
            const int64_t w = c0 + (int64_t)tid * R + r;
            if (off + need[r] > avail) {
                k.status[w] = ST_STATUS_DROPPED;
                pl->overflow = 1;
            } else {
                int64_t idx = base + snap + off;
                int32_t par = par0[r];
                const bool virt = par < 0;
                const float T = Tw[r];
                if (virt) {
                    // materialise the backward tree rooted at (q_g, T)
#pragma unroll
                    for (int jj = 0; jj < kMaxDof; ++jj)
                        if (jj < d) a.tree.x[(int64_t)jj * a.tree.total + idx] = a.sc.q_g[jj];
                    a.tree.x[(int64_t)d * a.tree.total + idx] = T;
                    a.tree.parent[idx] = -1;
                    a.tree.cost[idx] = 0.f;
                    a.tree.rootT[idx] = T;
                    atomicMin((int *)&pl->minRootT[p - 1], __float_as_int(T));
                    par = (int32_t)idx;
                    k.parent[w] = par;
                    ++idx;
                }
#pragma unroll
                for (int jj = 0; jj <= kMaxDof; ++jj)
                    if (jj <= d) a.tree.x[(int64_t)jj * a.tree.total + idx] = xv[r][jj];
                a.tree.parent[idx] = par;
                a.tree.cost[idx] = cn[r];
                a.tree.rootT[idx] = rn[r];
                k.new_idx[w] = (int32_t)idx;
                k.status[w] = ST_STATUS_ADVANCED;
                atomicMax(&s_last, (int)(off + need[r]));
                bset[r] = dr[r] == 0 ? 0 : 1;
            }
            off += need[r];
        }
        // the inserted workers are the bridge queries (a6): places within the
        // block from LDS counters, then one global atomic per set and pass
        int bpos[R];
#pragma unroll
        for (int r = 0; r < R; ++r) bpos[r] = wave_bucket_add(s_bcnt, bset[r]);
        __syncthreads();
        if (tid < 2) {
            const int c = s_bcnt[tid];
            s_bbase[tid] = c > 0 ? atomicAdd(&k.bcnt[kBcntBridge + tid], c) : 0;
            s_bcnt[tid] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (bset[r] >= 0)
                k.border_br[(int64_t)bset[r] * a.B + s_bbase[bset[r]] + bpos[r]] = (int32_t)(c0 + (int64_t)tid * R + r);
        // collided extensions (disjoint from the inserted workers), written
        // last so that no load of this pass waits behind them
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (trapped[r]) k.status[c0 + (int64_t)tid * R + r] = ST_STATUS_TRAPPED;
        running += s_total;
        __syncthreads();
    }
    if (tid == 0) pl->count[p] = (int32_t)(snap + s_last);
}

// ---------------------------------------------------------------------------
// a6: bridge selection merge
// ---------------------------------------------------------------------------


// Bridge selection's merge and the first states of the bridge edge in one
// launch, one wave per advanced worker, given densely (wave i takes the i-th
// worker of the bridge buckets, so the waves that check are packed into
// the first blocks and no SIMD holds more than one of them): the wave merges
// its worker's per-slice candidates (the lexicographic (key, index) minimum
// over the slices: arrival, then rho, then node index), then checks
// states 0 .. 63 of the chosen bridge edge (lane j takes state j, the FIRST
// rule over the wave), which decides every bridge that collides there or has
// at most 64 states.  The rest (no hit among 64 or more states) append their
// work items to the rank lists for the item kernel, which checks them whole.
// Wave i also writes the empty bridge of worker i when that worker did not
// advance.  The per-edge records (state count, least hit) are the plan
// step's; the finish step runs in the publish kernel.
template <int KIND, int OT, int OBS, bool MULTI>
__global__ __launch_bounds__(256) void k_bridge_check(BridgeArgs a0, EdgeArgs ea0, const BridgeArgs *__restrict__ av,
                                                      const EdgeArgs *__restrict__ ev,
                                                      const int32_t *__restrict__ members) {
    extern __shared__ float4 lds[];
    // many problems per launch: the member is blockIdx.x, so that members
    // vary fastest and every member's first blocks (the ones that check) are
    // dispatched ahead of the members' empty blocks; blocks past the
    // member's own grid leave
    const int bx = MULTI ? (int)blockIdx.y : (int)blockIdx.x;
    const int mi = MULTI ? members[blockIdx.x] : 0;
    const BridgeArgs &a = MULTI ? av[mi] : a0;
    const EdgeArgs &ea = MULTI ? ev[mi] : ea0;
    if (MULTI && (int64_t)bx * (blockDim.x >> 6) >= a.B) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = ((int64_t)bx * blockDim.x + threadIdx.x) >> 6;
    const Work &k = a.w;
    const SceneDev &sc = ea.sc;
    const EdgeBufs &eb = ea.eb;
    const int d = a.tree.d, W = d + 1;
    if (i < a.B && lane == 0 && k.status[i] != ST_STATUS_ADVANCED) {
        k.bridge[i] = -1;
        k.br_valid[i] = 0;
        k.Up[i] = INFINITY;
        k.Cp[i] = INFINITY;
        eb.n[i] = -1;
    }
    const int32_t nb0 = k.bcnt[kBcntBridge], nb1 = k.bcnt[kBcntBridge + 1];
    const int64_t nsel = (int64_t)nb0 + nb1;
    // a block past the advanced workers has nothing more to do (whole block)
    if ((int64_t)bx * (blockDim.x >> 6) >= nsel) return;
    const bool in = i < nsel;
    const int64_t w = in ? (i < nb0 ? k.border_br[i] : k.border_br[a.B + (i - nb0)]) : 0;
    unsigned long long bk = kNoKey;
    uint32_t bi = 0xffffffffu;
    if (in) {
        for (int y = lane; y < a.nch; y += 64) {
            const int32_t ii = k.br_idx[i * a.nch + y];
            if (ii < 0) continue;
            const unsigned long long kk = k.br_key[i * a.nch + y];
            if (kk < bk || (kk == bk && (uint32_t)ii < bi)) {
                bk = kk;
                bi = (uint32_t)ii;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long ok = __shfl_xor(bk, o, 64);
        const uint32_t oi = __shfl_xor(bi, o, 64);
        if (ok < bk || (ok == bk && oi < bi)) {
            bk = ok;
            bi = oi;
        }
    }
    const bool has = in && bi != 0xffffffffu;  // the same on every lane of the wave
    // the bridge's rows in flight while the block stages the scene
    float y[kMaxDof + 1], xn[kMaxDof + 1];
    float up = 0.f, cp = 0.f, cb = 0.f;
    if (has) {
#pragma unroll
        for (int j = 0; j <= kMaxDof; ++j) {
            y[j] = j <= d ? a.tree.x[(int64_t)j * a.tree.total + bi] : 0.f;
            xn[j] = j <= d ? k.xnew[w * W + j] : 0.f;
        }
        up = a.dir[w] == 0 ? a.tree.rootT[bi] : k.rootT_new[w];
        cp = k.cost_new[w];
        cb = a.tree.cost[bi];
    }
    stage_obstacles(sc, lds);
    if (!in) return;  // whole waves, after the block's barrier
    if (!has) {
        if (lane == 0) {
            k.bridge[w] = -1;
            k.br_valid[w] = 0;
            k.Up[w] = INFINITY;
            k.Cp[w] = INFINITY;
            eb.n[w] = -1;
        }
        return;
    }
    float D2 = 0.f;
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j) {
        if (j < d) {
            const float e = y[j] - xn[j];
            D2 = fmaf(e, e, D2);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j <= kMaxDof; ++j)
            if (j <= d) k.xb[w * W + j] = y[j];
        k.bridge[w] = (int32_t)bi;
        k.br_valid[w] = 1;
        k.Up[w] = up;
        k.Cp[w] = cp + sqrtf(D2) + cb;
    }
    // the edge (x_new, y), earlier time first, and its state count
    float A[kMaxDof + 1], B[kMaxDof + 1];
    const bool sw = xn[d] > y[d];
#pragma unroll
    for (int j = 0; j <= kMaxDof; ++j) {
        A[j] = sw ? y[j] : xn[j];
        B[j] = sw ? xn[j] : y[j];
    }
    const int32_t n = edge_states(A, B, d, sc.v_d, sc.h_d);
    const bool act = lane <= n;
    float q[kMaxDof];
    float t = 0.f;
    if (act && lane == n) {
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) q[j] = j < d ? B[j] : 0.f;
        t = B[d];
    } else if (act) {
        const float sj = (float)lane * (1.0f / (float)n);
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) q[j] = j < d ? fmaf(sj, B[j] - A[j], A[j]) : 0.f;
        t = fmaf(sj, B[d] - A[d], A[d]);
    } else {
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) q[j] = 0.f;
    }
    const bool hit = state_hits<KIND, OT, OBS, true>(sc, lds, q, t, act, ~0ull, (1ull << lane) - 1ull);
    const uint64_t hm = __ballot(hit && act);
    if (lane == 0) {
        eb.n[w] = n;
        eb.hit[w] = hm ? (int32_t)__builtin_ctzll(hm) : kNoHit;
    }
    if (hm || n < 64) return;  // decided
    // undecided: the whole edge goes to the item kernel (L states per chunk,
    // up to mmax items), one rank-list append per item
    const int L = 1 << (ea.lpe_shift - ea.split_shift);
    const int64_t c = ((int64_t)n + L) / L;
    const int m = (int)(c < eb.mmax ? c : eb.mmax);
    if (lane < m) {
        const int slot = atomicAdd(&eb.cnt[lane * kCntStride], 1);
        eb.items[(int64_t)lane * eb.cap + slot] = make_int2((int)w, lane);
    }
}

// ---------------------------------------------------------------------------
// a7: incumbent publish (lexicographic (U', C', worker) minimum)
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// a8 / a9: allocation update after a strict drop of U
// ---------------------------------------------------------------------------


// Runs at the end of the publish block: every thread of the block calls it,
// after a barrier that makes the incumbent update visible.
__device__ __forceinline__ void roots_body(const RootsArgs &a) {
    __shared__ int cand[kMaxGroups], assign[kMaxGroups], donor[kMaxGroups];
    __shared__ int s_kend;
    PlanDev *pl = a.pl;
    if (pl->improved != 2) return;
    const int tid = threadIdx.x, N = a.N;
    const WindowsDev &w = a.win;
    if (a.variant == ST_INTERVAL_ROOT) {
        // repartition below Ubar = min(H, U); trees rooted at T >= U drop out
        // of the scans through their root time
        if (tid == 0) {
            const double Ubar = fmin(w.H, (double)pl->U);
            int j = 0;
            int lo = 0, hi = w.nw;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (w.lo[mid] < Ubar) lo = mid + 1;
                else hi = mid;
            }
            j = lo;
            pl->Ubar = Ubar;
            pl->jstar = j;
            pl->G = j > 0 ? w.cum[j - 1] + (fmin(w.hi[j - 1], Ubar) - w.lo[j - 1]) : 0.0;
            pl->done = !(w.L < Ubar);
        }
        return;
    }
    const float U = pl->U;
    if (tid < N) {
        const float T = pl->slotT[tid];
        if (T >= U) pl->slot_active[tid] = 0;
        donor[tid] = T > U ? 1 : 0;
        assign[tid] = -1;
    }
    if (tid == 0) {
        // first grid index whose time (as stored) is not below U
        int k = w.k_lo;
        while (k <= w.k_hi && (float)((double)k * w.dt) < U) ++k;
        s_kend = k;
    }
    __syncthreads();
    // the no-recycling ablation keeps the initial roots: deactivation only
    const int64_t K = a.no_recycling ? 0 : s_kend - w.k_lo;
    if (tid < N && K > 0) {
        const int64_t a0 = w.k_lo + (K * tid) / N, b0 = w.k_lo + (K * (tid + 1)) / N;
        bool occupied = false;
        for (int s = 0; s < N; ++s)
            if (pl->slot_active[s] && pl->slotK[s] >= a0 && pl->slotK[s] < b0) occupied = true;
        int c = -1;
        if (!occupied)
            for (int64_t k = a0; k < b0; ++k)
                if (w.gfree[k - w.k_lo]) {
                    c = (int)k;
                    break;
                }
        cand[tid] = c;
    } else if (tid < N) {
        cand[tid] = -1;
    }
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int st_ = 0; st_ < N; ++st_) {
            if (cand[st_] < 0) continue;
            while (s < N && !donor[s]) ++s;
            if (s >= N) break;
            assign[s++] = cand[st_];
        }
    }
    __syncthreads();
    if (tid < N && assign[tid] >= 0) {
        const int s = tid;
        const int k = assign[s];
        const float T = (float)((double)k * w.dt);
        const int64_t idx = pool_base(a.tree, 1 + s);
        for (int j = 0; j < a.sc.d; ++j) a.tree.x[(int64_t)j * a.tree.total + idx] = a.sc.q_g[j];
        a.tree.x[(int64_t)a.sc.d * a.tree.total + idx] = T;
        a.tree.parent[idx] = -1;
        a.tree.cost[idx] = 0.f;
        a.tree.rootT[idx] = T;
        pl->count[1 + s] = 1;
        pl->slot_gen[s] += 1;
        pl->slotT[s] = T;
        pl->slotK[s] = k;
        pl->slot_active[s] = 1;
    }
    __syncthreads();
    if (tid == 0) {
        int na = 0;
        for (int s = 0; s < N; ++s)
            if (pl->slot_active[s]) pl->active_list[na++] = s;
        pl->n_active = na;
    }
}

__device__ __forceinline__ bool lex_less(float u1, float c1, int w1, float u2, float c2, int w2) {
    if (u1 != u2) return u1 < u2;
    if (c1 != c2) return c1 < c2;
    return (uint32_t)w1 < (uint32_t)w2;
}

template <bool MULTI>
__global__ __launch_bounds__(1024) void k_publish(PublishArgs a0, const PublishArgs *__restrict__ av, RootsArgs r0,
                                                  const RootsArgs *__restrict__ rv) {
    __shared__ float sU[16], sC[16];  // one candidate per wave (1024 threads)
    __shared__ int sW[16];
    const PublishArgs &a = MULTI ? av[blockIdx.y] : a0;
    const int tid = threadIdx.x;
    const Work &k = a.w;
    float bu = INFINITY, bc = INFINITY;
    int bw = -1;
    unsigned long long states = 0, edges = 0;
    // No global store before the last load of this pass (a store ahead of a
    // load makes the load's wait include the store's completion): the bridge
    // finish step (free / first hit, work counters) and the incumbent
    // candidates read the workers' records; the outputs are written below.
    for (int64_t w = tid; w < a.B; w += blockDim.x) {
        const bool bv = k.br_valid[w];
        const int8_t st = k.status[w];
        const int32_t h = a.eb.hit[w];
        const int32_t n = a.eb.n[w];
        const float up = k.Up[w], cp = k.Cp[w];
        const bool bfree = bv && h == kNoHit;
        if (bv) {
            // algorithmic work: the states up to the first hit, all n+1 when free
            states += bfree ? (unsigned long long)n + 1ull : (unsigned long long)h + 1ull;
            edges += 1;
        }
        if (st == ST_STATUS_ADVANCED && bfree && lex_less(up, cp, (int)w, bu, bc, bw)) {
            bu = up;
            bc = cp;
            bw = (int)w;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        states += __shfl_down(states, o, 64);
        edges += __shfl_down(edges, o, 64);
    }
    // the lexicographic minimum: within each wave by shuffles, then over the
    // waves' results by wave 0 (every lane of a wave ends with its minimum)
    auto wave_min = [&](float &u, float &c, int &wk) {
        for (int o = 32; o > 0; o >>= 1) {
            const float ou = __shfl_xor(u, o, 64), oc = __shfl_xor(c, o, 64);
            const int ow = __shfl_xor(wk, o, 64);
            if (lex_less(ou, oc, ow, u, c, wk)) {
                u = ou;
                c = oc;
                wk = ow;
            }
        }
    };
    wave_min(bu, bc, bw);
    const int nwv = (int)(blockDim.x >> 6);
    if ((tid & 63) == 0) {
        sU[tid >> 6] = bu;
        sC[tid >> 6] = bc;
        sW[tid >> 6] = bw;
    }
    __syncthreads();
    if (tid < 64) {
        float u = tid < nwv ? sU[tid] : INFINITY, c = tid < nwv ? sC[tid] : INFINITY;
        int wk = tid < nwv ? sW[tid] : -1;
        wave_min(u, c, wk);
        if (tid == 0) {
            sU[0] = u;
            sC[0] = c;
            sW[0] = wk;
        }
    }
    __syncthreads();
    if (tid == 0) {
        PlanDev *pl = a.pl;
        const int w = sW[0];
        // every load before the first store
        const float U0 = pl->U, C0 = pl->C;
        const int32_t it = pl->iter, fi = pl->first_iter;
        int8_t dw = 0;
        int32_t ni = -1, bw = -1;
        if (w >= 0) {
            dw = a.dir[w];
            ni = k.new_idx[w];
            bw = k.bridge[w];
        }
        if (w >= 0 && (sU[0] < U0 || (sU[0] == U0 && sC[0] < C0))) {
            pl->improved = sU[0] < U0 ? 2 : 1;
            pl->U = sU[0];
            pl->C = sC[0];
            pl->inc_f = dw == 0 ? ni : bw;
            pl->inc_b = dw == 0 ? bw : ni;
            if (fi < 0) pl->first_iter = it;
        }
        pl->iter = it + 1;
    }
    if ((tid & 63) == 0 && edges) {
        atomicAdd(&a.work_br[0], edges);
        atomicAdd(&a.work_br[1], states);
    }
    // the rank lists of the edge pipeline and the bridge buckets are consumed:
    // empty for the next launch
    if (tid < a.eb.mmax) a.eb.cnt[tid * kCntStride] = 0;
    if (tid < 2) k.bcnt[kBcntBridge + tid] = 0;
    // optional caller outputs (a candidate that is not a free bridge of an
    // advanced worker reports U = C = infinity)
    const st_extend_out &o = a.out;
    if (o.status || o.parent || o.new_idx || o.bridge || o.bridge_ok || o.Up || o.Cp) {
        for (int64_t w = tid; w < a.B; w += blockDim.x) {
            const int8_t st = k.status[w];
            const bool bv = k.br_valid[w];
            const bool bfree = bv && a.eb.hit[w] == kNoHit;
            const bool ok = st == ST_STATUS_ADVANCED && bfree;
            if (o.status) o.status[w] = st;
            if (o.parent) o.parent[w] = k.parent[w];
            if (o.new_idx) o.new_idx[w] = k.new_idx[w];
            if (o.bridge) o.bridge[w] = k.bridge[w];
            if (o.bridge_ok) o.bridge_ok[w] = ok ? 1 : 0;
            if (o.Up) o.Up[w] = ok ? k.Up[w] : INFINITY;
            if (o.Cp) o.Cp[w] = ok ? k.Cp[w] : INFINITY;
        }
    }
    // a8 / a9 in the same block (no launch of its own)
    __syncthreads();
    roots_body(MULTI ? rv[blockIdx.y] : r0);
}

struct XnewOutArgs {
    int64_t B;
    int32_t d;
    const int8_t *status;
    const float *xnew;
    float *out;
};

__global__ void k_xnew_out(XnewOutArgs a) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.B) return;
    const bool adv = a.status[w] >= ST_STATUS_ADVANCED;
    for (int j = 0; j <= a.d; ++j) a.out[(int64_t)j * a.B + w] = adv ? a.xnew[w * (a.d + 1) + j] : 0.f;
}

// ---------------------------------------------------------------------------
// learned proposal parameters from the network output z
// ---------------------------------------------------------------------------

__global__ void k_prop_set(PlanDev *pl, const float *z, float mix) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!z || !(mix > 0.f)) {
        pl->prop_mix = 0.f;
        return;
    }
    float mx = -INFINITY;
    for (int c = 0; c < 8; ++c) mx = fmaxf(mx, z[c]);
    float s = 0.f;
    for (int c = 0; c < 8; ++c) s += expf(z[c] - mx);
    float acc = 0.f;
    for (int c = 0; c < 8; ++c) {
        acc += expf(z[c] - mx) / s;
        pl->prop_wcum[c] = acc;
    }
    pl->prop_wcum[7] = 1.f;
    for (int i = 0; i < 64; ++i) {
        pl->prop_mu[i] = z[8 + i];
        pl->prop_sd[i] = expf(z[72 + i]);
    }
    mx = -INFINITY;
    for (int b = 0; b < 32; ++b) mx = fmaxf(mx, z[136 + b]);
    s = 0.f;
    for (int b = 0; b < 32; ++b) s += expf(z[136 + b] - mx);
    acc = 0.f;
    for (int b = 0; b < 32; ++b) {
        acc += expf(z[136 + b] - mx) / s;
        pl->prop_hcum[b] = acc;
    }
    pl->prop_hcum[31] = 1.f;
    pl->prop_mix = mix;
}

// ---------------------------------------------------------------------------
// nearest-node results for the C ABI
// ---------------------------------------------------------------------------

__global__ void k_nn_out(int64_t M, int metric, const unsigned long long *keys, int32_t *idx, float *dist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const unsigned long long k = keys[i];
    const bool none = k == kNoKey;
    idx[i] = none ? -1 : (int32_t)(k & 0xffffffffu);
    if (dist) {
        const float kf = __uint_as_float((uint32_t)(k >> 32));
        dist[i] = none ? INFINITY : (metric == ST_METRIC_RHO ? sqrtf(0.5f * kf) : sqrtf(kf));
    }
}

__global__ void k_fill_tiles(int64_t M, int set, int sigma, int4 *tiles, int32_t *n_tiles, unsigned long long *keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nt = (M + kTileQ - 1) / kTileQ;
    if (i < nt) tiles[i] = make_int4(set, (int)(i * kTileQ), (int)min<int64_t>(kTileQ, M - i * kTileQ), sigma);
    if (i == 0) n_tiles[0] = (int32_t)nt;
    for (int64_t j = i; j < M; j += (int64_t)gridDim.x * blockDim.x) keys[j] = kNoKey;
}

// ---------------------------------------------------------------------------
// path extraction and timestamps
// ---------------------------------------------------------------------------

// Lengths of the incumbent's forward chain (v_f back to the root) and
// backward chain (w_b to its root).  A chain only points to earlier nodes of
// its own pool, so it cannot be longer than that pool's node count; a longer
// walk means a corrupted tree and is reported as -1.
__global__ void k_path_len(TreeDev tree, const PlanDev *pl, int32_t *len_out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int32_t f = pl->inc_f, b = pl->inc_b;
    len_out[0] = len_out[1] = 0;
    if (f < 0 || b < 0) return;
    const int32_t heads[2] = {f, b};
    for (int c = 0; c < 2; ++c) {
        const int64_t limit = tree.total;
        int64_t n = 0;
        for (int32_t i = heads[c]; i >= 0 && n <= limit; i = tree.parent[i]) ++n;
        len_out[c] = n > limit ? -1 : (int32_t)n;
    }
}

// The incumbent path into out[(nf + nb)][d+1]: the forward chain written back
// to front (root first), then the backward chain from w_b to its root.
__global__ void k_path_copy(TreeDev tree, const PlanDev *pl, int32_t nf, int32_t nb, float *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int d = tree.d, W = d + 1;
    int32_t i = pl->inc_f;
    for (int j = nf - 1; j >= 0 && i >= 0; --j, i = tree.parent[i])
        for (int c = 0; c <= d; ++c) out[(int64_t)j * W + c] = tree.x[(int64_t)c * tree.total + i];
    i = pl->inc_b;
    for (int j = nf; j < nf + nb && i >= 0; ++j, i = tree.parent[i])
        for (int c = 0; c <= d; ++c) out[(int64_t)j * W + c] = tree.x[(int64_t)c * tree.total + i];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int V>
using IC = std::integral_constant<int, V>;

static int ot_for(int O_pad) {
    if (O_pad <= 4) return 4;
    if (O_pad <= 8) return 8;
    return 16;
}

template <class F>
static void dispatch_scene2(const SceneDev &sc, F &&f);

// The edge-check kernels' instance for a scene: as dispatch_scene2, with an
// arm that has static geometry as kDHStatic.
template <class F>
static void dispatch_scene_edges(const SceneDev &sc, F &&f) {
    if (sc.kind != kTranslate && sc.stat) {
        auto by_ot = [&](auto obs) {
            switch (sc.ot) {
                case 4: f(IC<kDHStatic>{}, IC<4>{}, obs); break;
                case 8: f(IC<kDHStatic>{}, IC<8>{}, obs); break;
                default: f(IC<kDHStatic>{}, IC<16>{}, obs); break;
            }
        };
        if (sc.obs_mode == kObsShared) by_ot(IC<kObsShared>{});
        else by_ot(IC<kObsGeneric>{});
        return;
    }
    dispatch_scene2(sc, f);
}

template <class F>
static void dispatch_scene2(const SceneDev &sc, F &&f) {
    auto by_ot = [&](auto kind, auto obs) {
        switch (sc.ot) {
            case 4: f(kind, IC<4>{}, obs); break;
            case 8: f(kind, IC<8>{}, obs); break;
            default: f(kind, IC<16>{}, obs); break;
        }
    };
    auto by_obs = [&](auto kind) {
        if (sc.obs_mode == kObsShared) by_ot(kind, IC<kObsShared>{});
        else by_ot(kind, IC<kObsGeneric>{});
    };
    if (sc.kind == kTranslate) by_obs(IC<kTranslate>{});
    else by_obs(IC<kDH>{});
}

template <class T>
static hipError_t dalloc(T **p, size_t n) {
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

void work_free(st_problem *p) {
    Work &w = p->work;
    void *bufs[] = {w.dir, w.flags, w.grp, w.T, w.qr, w.tr, w.nn_key, w.tiles, w.n_tiles, w.bcnt, w.border_nn,
                    w.border_br, w.xn, w.xnew, w.edge_valid, w.edge_free, w.first_hit, w.status, w.parent, w.new_idx, w.cost_new,
                    w.rootT_new, w.br_key, w.br_idx, w.bridge, w.xb, w.br_valid, w.br_free, w.Up, w.Cp};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    memset(&w, 0, sizeof w);
}

static int max_tiles(int64_t B, int n_sets) { return (int)((B + kTileQ - 1) / kTileQ) + n_sets; }
int max_query_tiles(int64_t B, int n_sets) { return max_tiles(B, n_sets); }

int work_reserve(st_problem *p, int64_t B) {
    if (p->work.Bcap >= B) return ST_OK;
    ST_HIP(hipDeviceSynchronize());
    graphs_free(p);
    work_free(p);
    Work &w = p->work;
    const int W = p->d + 1;
    const int mt = max_tiles(B, p->tree.n_pools + 2);
    w.Bcap = B;
    ST_HIP(dalloc(&w.dir, B));
    ST_HIP(dalloc(&w.flags, B));
    ST_HIP(dalloc(&w.grp, B));
    ST_HIP(dalloc(&w.T, B));
    ST_HIP(dalloc(&w.qr, (size_t)B * p->d));
    ST_HIP(dalloc(&w.tr, B));
    ST_HIP(dalloc(&w.nn_key, B));
    ST_HIP(dalloc(&w.bcnt, kBcntSize));
    ST_HIP(dalloc(&w.border_nn, (size_t)p->tree.n_pools * B));
    ST_HIP(dalloc(&w.border_br, (size_t)2 * B));
    ST_HIP(dalloc(&w.tiles, (size_t)mt * 4));
    ST_HIP(dalloc(&w.n_tiles, 4));
    ST_HIP(dalloc(&w.xn, (size_t)B * W));
    ST_HIP(dalloc(&w.xnew, (size_t)B * W));
    ST_HIP(dalloc(&w.edge_valid, B));
    ST_HIP(dalloc(&w.edge_free, B));
    ST_HIP(dalloc(&w.first_hit, B));
    ST_HIP(dalloc(&w.status, B));
    ST_HIP(dalloc(&w.parent, B));
    ST_HIP(dalloc(&w.new_idx, B));
    ST_HIP(dalloc(&w.cost_new, B));
    ST_HIP(dalloc(&w.rootT_new, B));
    ST_HIP(dalloc(&w.br_key, (size_t)kMaxNch * B));
    ST_HIP(dalloc(&w.br_idx, (size_t)kMaxNch * B));
    ST_HIP(dalloc(&w.bridge, B));
    ST_HIP(dalloc(&w.xb, (size_t)B * W));
    ST_HIP(dalloc(&w.br_valid, B));
    ST_HIP(dalloc(&w.br_free, B));
    ST_HIP(dalloc(&w.Up, B));
    ST_HIP(dalloc(&w.Cp, B));
    ST_HIP(hipMemset(w.bcnt, 0, kBcntSize * sizeof(int32_t)));
    ST_HIP(hipMemset(w.edge_free, 0, B));
    ST_HIP(hipMemset(w.br_free, 0, B));
    return ST_OK;
}

// Node slices per tile: about `blocks` scan blocks in all.  More slices cut
// the nodes one thread walks (the latency of a scan of a large tree) but
// add partial results: the nearest-node scan merges them with 64-bit atomics
// (one per query and slice), the bridge scan with a per-worker reduction.
static int nch_for(int tiles, int blocks = 1024) {
    int n = blocks / std::max(tiles, 1);
    return std::max(1, std::min(kMaxNch, n));
}
int nch_for_tiles(int tiles) { return nch_for(tiles); }

void prof_mark(st_problem *p, int stage, hipStream_t s) {
    if (!p->prof) return;
    if (p->prof_used == p->prof_ev.size()) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return;
        p->prof_ev.push_back(ev);
        p->prof_stage.push_back(0);
    }
    p->prof_stage[p->prof_used] = stage;
    (void)hipEventRecord(p->prof_ev[p->prof_used], s);
    p->prof_used++;
}

SampleArgs make_sample_args(const st_problem *p, int64_t iter, int64_t B, const st_samples &out, bool bucket) {
    SampleArgs a;
    memset(&a, 0, sizeof a);
    a.sc = p->sc;
    a.win = p->win;
    a.pl = p->d_plan;
    a.variant = p->prm.variant;
    a.N = p->prm.n_groups;
    a.p_guided = (float)p->prm.p_guided;
    a.p_new = (float)p->prm.p_new;
    a.seed = p->prm.seed;
    a.pid = p->prm.problem_id;
    a.iter = iter;
    a.B = B;
    a.t_min = p->t_min;
    a.t_max = p->t_max;
    a.out = out;
    a.nb = (int)((B * (p->sc.kind == kTranslate ? 1 : sample_lanes<kDH>()) + 255) / 256);
    (void)sample_lds_bytes(p, &a.nw_lds);
    a.n_pools = p->tree.n_pools;
    a.bcnt = bucket ? p->work.bcnt : nullptr;
    a.border = bucket ? p->work.border_nn : nullptr;
    a.keys = bucket ? p->work.nn_key : nullptr;
    return a;
}

size_t sample_lds_bytes(const st_problem *p, int32_t *nw_lds) {
    const size_t scene = scene_lds_bytes(p->sc);
    const int32_t nw = p->prm.variant == ST_INTERVAL_ROOT ? p->win.nw : 0;
    // windows are staged while the whole stays within 64 KB of LDS
    const bool fit = scene + (size_t)nw * 3 * sizeof(double) <= 64 * 1024;
    if (nw_lds) *nw_lds = fit ? nw : 0;
    return scene + (fit ? (size_t)nw * 3 * sizeof(double) : 0);
}

int sample_batch(st_problem *p, int64_t iter, int64_t B, const st_samples &out, hipStream_t s, bool bucket) {
    prof_mark(p, kStSample, s);
    const SampleArgs a = make_sample_args(p, iter, B, out, bucket);
    const size_t lds = sample_lds_bytes(p, nullptr);
    dispatch_scene2(p->sc, [&](auto kind, auto ot, auto obs) {
        k_sample<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, false>
            <<<dim3(a.nb), dim3(256), lds, s>>>(a, nullptr, nullptr);
    });
    ST_HIP(hipGetLastError());
    return ST_OK;
}

static int edge_shift(const st_problem *p, bool bridge) { return bridge ? p->tune_br : p->tune_ext; }

void make_iter_args(const st_problem *p, int64_t B, const st_samples &in, const st_extend_out *out, int nch_nn,
                    int nch_br, int min_item_blocks, int64_t launch_edges, IterArgs &a) {
    const Work &w = p->work;
    const int np = p->tree.n_pools;
    const int d = p->d;
    // snapshot + buckets for the nearest-node scans (a2)
    PrepArgs &pa = a.prep_nn;
    memset(&pa, 0, sizeof pa);
    pa.pl = p->d_plan;
    pa.variant = p->prm.variant;
    pa.n_pools = np;
    pa.d = d;
    pa.B = B;
    pa.s = in;
    pa.bcnt = w.bcnt;
    pa.border = w.border_nn;
    pa.keys = w.nn_key;
    a.mt_nn = max_tiles(B, np);
    ScanArgs &sa = a.scan_nn;
    memset(&sa, 0, sizeof sa);
    sa.tree = p->tree;
    sa.pl = p->d_plan;
    sa.use_snap = 1;
    sa.variant = p->prm.variant;
    sa.v = p->sc.v;
    // the samples themselves (SoA) are the queries
    sa.qx = in.qr;
    sa.sq = 1;
    sa.sj = B;
    sa.qt = in.tr;
    sa.st = 1;
    sa.bmode = 1;
    sa.bcnt = w.bcnt;
    sa.border = w.border_nn;
    sa.bstride = B;
    sa.keys = w.nn_key;
    sa.nch = nch_nn;
    // steering (a3)
    SteerArgs &ta = a.steer;
    ta.sc = p->sc;
    ta.tree = p->tree;
    ta.pl = p->d_plan;
    ta.variant = p->prm.variant;
    ta.eta = (float)p->prm.eta;
    ta.B = B;
    ta.s = in;
    ta.w = w;
    // extension edge checks (a4)
    a.edge_ext = edge_args(p->sc, p->ebufs, B, w.xn, w.xnew, w.edge_valid, w.edge_free, w.first_hit,
                           edge_shift(p, false), p->d_plan->work, min_item_blocks,
                           split_for(p->split_ext, launch_edges));
    // extension edges are short (rho <= eta: at most ceil(sqrt(2) eta / h) + 1
    // states): the flattened path, unless eta / h is unusually large
    a.edge_ext.flat = std::sqrt(2.0) * p->prm.eta / p->prm.h <= 4096.0 ? p->flat_ext : 0;
    // insertion (a5)
    InsertArgs &ia = a.insert;
    ia.sc = p->sc;
    ia.tree = p->tree;
    ia.pl = p->d_plan;
    ia.variant = p->prm.variant;
    ia.B = B;
    ia.s = in;
    ia.w = w;
    // bridges (a6)
    a.mt_br = max_tiles(B, 2);
    ScanArgs &sb = a.scan_br;
    sb = sa;
    // the new nodes (AoS [B][d+1]) are the queries
    sb.qx = w.xnew;
    sb.sq = d + 1;
    sb.sj = 1;
    sb.qt = w.xnew + d;
    sb.st = d + 1;
    sb.bmode = 2;
    sb.bcnt = w.bcnt + kBcntBridge;
    sb.border = w.border_br;
    sb.keys = nullptr;
    sb.pkey = w.br_key;
    sb.pidx = w.br_idx;
    sb.pstride = nch_br;  // query-major partials: [bridge query in bucket order][slice]
    sb.nch = nch_br;
    BridgeArgs &ba = a.merge;
    ba.tree = p->tree;
    ba.B = B;
    ba.nch = nch_br;
    ba.dir = in.dir;
    ba.w = w;
    a.edge_br = edge_args(p->sc, p->ebufs, B, w.xnew, w.xb, w.br_valid, w.br_free, w.first_hit, edge_shift(p, true),
                          p->d_plan->work + 2, min_item_blocks, split_for(p->split_br, launch_edges));
    a.edge_br.skip_finish = 1;  // k_publish reads the bridge hits itself
    // publish (a7)
    PublishArgs &pb = a.publish;
    pb.pl = p->d_plan;
    pb.B = B;
    pb.dir = in.dir;
    pb.w = w;
    if (out) pb.out = *out;
    else memset(&pb.out, 0, sizeof pb.out);
    pb.eb = p->ebufs;
    pb.work_br = p->d_plan->work + 2;
    // allocation update (a8 / a9)
    RootsArgs &ra = a.roots;
    ra.sc = p->sc;
    ra.tree = p->tree;
    ra.win = p->win;
    ra.pl = p->d_plan;
    ra.variant = p->prm.variant;
    ra.N = p->prm.n_groups;
    ra.no_recycling = p->prm.no_recycling;
}

int extend_batch(st_problem *p, int64_t B, const st_samples &in, const st_extend_out *out, hipStream_t s,
                 bool bucketed) {
    int rc = work_reserve(p, B);
    if (rc != ST_OK) return rc;
    if (p->ebufs.cap < B) {
        graphs_free(p);
        if ((rc = edge_bufs_reserve(p->ebufs, B)) != ST_OK) return rc;
    }
    IterArgs a;
    // node slices per scan tile: a budget of 4096 blocks for the nearest-node
    // scan, 1024 for the bridge scan (its per-slice candidates are merged by
    // the bridge check, which reads one per slice)
    make_iter_args(p, B, in, out, nch_for(max_tiles(B, p->tree.n_pools), 4096), nch_for(max_tiles(B, 2), 1024), 1024,
                   B, a);
    const int blocks = (int)((B + 255) / 256);
    prof_mark(p, kStNearest, s);
    if (!bucketed) {
        k_prep<<<1, 1024, 0, s>>>(a.prep_nn);
        ST_HIP(hipGetLastError());
    }
    if (p->prm.variant == ST_INTERVAL_ROOT)
        k_scan<kScanRho, false><<<dim3(a.mt_nn, a.scan_nn.nch), kTileQ, 0, s>>>(a.scan_nn, nullptr, nullptr);
    else
        k_scan<kScanConfig, false><<<dim3(a.mt_nn, a.scan_nn.nch), kTileQ, 0, s>>>(a.scan_nn, nullptr, nullptr);
    ST_HIP(hipGetLastError());
    if (a.edge_ext.flat) {
        // steering (a3) inside the extension check's launch (a4); the stage
        // timing counts the launch as the edge check
        prof_mark(p, kStEdge, s);
        const EdgeArgs &ea = a.edge_ext;
        dispatch_scene_edges(p->sc, [&](auto kind, auto ot, auto obs) {
            k_steer_flat<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value>
                <<<dim3(flat_blocks(ea.E, ea.flat)), dim3(64 * kFlatWaves), scene_lds_bytes(p->sc), s>>>(a.steer,
                                                                                                          ea);
        });
        ST_HIP(hipGetLastError());
    } else {
        prof_mark(p, kStSteer, s);
        k_steer<false><<<blocks, 256, 0, s>>>(a.steer, nullptr);
        ST_HIP(hipGetLastError());
        prof_mark(p, kStEdge, s);
        ST_HIP(launch_edge_args(a.edge_ext, s));
    }
    prof_mark(p, kStInsert, s);
    k_insert<false><<<p->tree.n_pools, insert_threads(B), 0, s>>>(a.insert, nullptr);
    ST_HIP(hipGetLastError());
    prof_mark(p, kStBridgeSel, s);
    k_scan<kScanBridge, false><<<dim3(a.mt_br, a.scan_br.nch), kTileQ, 0, s>>>(a.scan_br, nullptr, nullptr);
    ST_HIP(hipGetLastError());
    // the merge and the first 64 states of every bridge edge in one launch
    // (its stage timing counts it as the bridge check), then the item kernel
    // for the undecided rest
    prof_mark(p, kStBridgeEdge, s);
    dispatch_scene_edges(p->sc, [&](auto kind, auto ot, auto obs) {
        k_bridge_check<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, false>
            <<<(int)((B * 64 + 255) / 256), 256, scene_lds_bytes(p->sc), s>>>(a.merge, a.edge_br, nullptr, nullptr,
                                                                             nullptr);
    });
    ST_HIP(hipGetLastError());
    ST_HIP(launch_edge_items(a.edge_br, s));
    prof_mark(p, kStPublish, s);
    k_publish<false><<<1, 1024, 0, s>>>(a.publish, nullptr, a.roots, nullptr);
    ST_HIP(hipGetLastError());
    if (out && out->xnew) {
        XnewOutArgs xa{B, p->d, p->work.status, p->work.xnew, out->xnew};
        k_xnew_out<<<blocks, 256, 0, s>>>(xa);
        ST_HIP(hipGetLastError());
    }
    prof_mark(p, kStEnd, s);
    return ST_OK;
}

// ---------------------------------------------------------------------------
// many problems per launch: one iteration of every problem of a batch
// ---------------------------------------------------------------------------

int launch_batch_iteration(const BatchLaunch &L, hipStream_t s) {
    for (const BatchClass &c : L.classes) {
        dispatch_scene2(c.key, [&](auto kind, auto ot, auto obs) {
            k_sample<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, true>
                <<<dim3(c.nb_sample, c.n), dim3(256), c.lds_sample, s>>>(SampleArgs{}, L.sample, c.members);
        });
    }
    ST_HIP(hipGetLastError());
    auto scan_multi = [&](auto mode, auto tq, int mt, int n, const int32_t *members, const ScanArgs *args) {
        k_scan<decltype(mode)::value, true, decltype(tq)::value>
            <<<dim3(mt, L.nch, n), decltype(tq)::value, 0, s>>>(ScanArgs{}, args, members);
    };
    auto scan_launch = [&](auto mode, int mt, int n, const int32_t *members, const ScanArgs *args) {
        if (L.scan_tq == 64) scan_multi(mode, IC<64>{}, mt, n, members, args);
        else scan_multi(mode, IC<kTileQ>{}, mt, n, members, args);
    };
    if (L.n_ir > 0) scan_launch(IC<kScanRho>{}, L.mt_nn_ir, L.n_ir, L.ir_members, L.scan_nn);
    if (L.n_rr > 0) scan_launch(IC<kScanConfig>{}, L.mt_nn_rr, L.n_rr, L.rr_members, L.scan_nn);
    if (L.ext_flat) {
        // steering inside the flattened extension check, per scene class
        for (const BatchClass &c : L.classes) {
            dispatch_scene_edges(c.key, [&](auto kind, auto ot, auto obs) {
                k_steer_flat_multi<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value>
                    <<<dim3(c.nb_flat, c.n), dim3(64 * kFlatWaves), c.lds, s>>>(L.steer, L.edge_ext, c.members);
            });
            ST_HIP(hipGetLastError());
        }
    } else {
        k_steer<true><<<dim3(L.nb_worker, L.P), 256, 0, s>>>(SteerArgs{}, L.steer);
        ST_HIP(hipGetLastError());
        ST_HIP(launch_edge_plan_multi(L.edge_ext, L.P, L.nb_edge, s));
        for (const BatchClass &c : L.classes)
            ST_HIP(launch_edge_items_multi(c.key, c.split_ext, L.edge_ext, c.members, c.n, c.nb_items_ext, c.lds, s));
        ST_HIP(launch_edge_finish_multi(L.edge_ext, L.P, L.nb_edge, s));
    }
    k_insert<true><<<dim3(L.max_pools, L.P), L.ins_threads, 0, s>>>(InsertArgs{}, L.insert);
    scan_launch(IC<kScanBridge>{}, L.mt_br, L.P, L.all_members, L.scan_br);
    // the merge and the first 64 states of every bridge edge, per scene
    // class, then the item kernel for the undecided rest; one wave per block
    // (a member's blocks past its advanced workers leave before staging, and
    // a checking wave does not wait for three others to be scheduled)
    for (const BatchClass &c : L.classes) {
        dispatch_scene_edges(c.key, [&](auto kind, auto ot, auto obs) {
            k_bridge_check<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, true>
                <<<dim3(c.n, c.nb_bcheck), 64, c.lds, s>>>(BridgeArgs{}, EdgeArgs{}, L.merge, L.edge_br, c.members);
        });
        ST_HIP(hipGetLastError());
    }
    for (const BatchClass &c : L.classes)
        ST_HIP(launch_edge_items_multi(c.key, c.split_br, L.edge_br, c.members, c.n, c.nb_items_br, c.lds, s));
    k_publish<true><<<dim3(1, L.P), 1024, 0, s>>>(PublishArgs{}, L.publish, RootsArgs{}, L.roots);
    ST_HIP(hipGetLastError());
    return ST_OK;
}

int nearest_set(st_problem *p, int32_t set, int32_t metric, int32_t sigma, int64_t M, const float *xq,
                int32_t *idx_out, float *dist_out, hipStream_t s) {
    if (M <= 0) return ST_OK;
    int rc = work_reserve(p, M);
    if (rc != ST_OK) return rc;
    Work &w = p->work;
    const int nt = (int)((M + kTileQ - 1) / kTileQ);
    k_fill_tiles<<<(nt + 255) / 256, 256, 0, s>>>(M, set < 0 ? (set == ST_SET_FORWARD ? 0 : kSetAllBackward) : 1 + set,
                                                 sigma, (int4 *)w.tiles, w.n_tiles, w.nn_key);
    ST_HIP(hipGetLastError());
    ScanArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.tree = p->tree;
    sa.pl = p->d_plan;
    sa.use_snap = 0;
    sa.variant = p->prm.variant;
    sa.v = p->sc.v;
    sa.qx = xq;
    sa.sq = p->d + 1;
    sa.sj = 1;
    sa.qt = xq + p->d;
    sa.st = p->d + 1;
    sa.bmode = 0;
    sa.tiles = (const int4 *)w.tiles;
    sa.n_tiles = w.n_tiles;
    sa.keys = w.nn_key;
    sa.nch = nch_for(nt);
    if (metric == ST_METRIC_RHO) k_scan<kScanRho, false><<<dim3(nt, sa.nch), kTileQ, 0, s>>>(sa, nullptr, nullptr);
    else k_scan<kScanConfig, false><<<dim3(nt, sa.nch), kTileQ, 0, s>>>(sa, nullptr, nullptr);
    ST_HIP(hipGetLastError());
    k_nn_out<<<(int)((M + 255) / 256), 256, 0, s>>>(M, metric, w.nn_key, idx_out, dist_out);
    ST_HIP(hipGetLastError());
    return ST_OK;
}

static st_samples work_samples(st_problem *p) {
    Work &w = p->work;
    st_samples s;
    s.dir = w.dir;
    s.flags = w.flags;
    s.grp = w.grp;
    s.T = w.T;
    s.qr = w.qr;
    s.tr = w.tr;
    return s;
}

st_samples work_samples_of(st_problem *p) { return work_samples(p); }

void graphs_free(st_problem *p) {
    for (int k = 0; k < 2; ++k) {
        if (p->graph[k]) (void)hipGraphExecDestroy(p->graph[k]);
        p->graph[k] = nullptr;
    }
    p->graph_B = 0;
}

// Capture `n` iterations (sample + extend batch, all kernels) into an
// executable graph on the problem's capture stream.  The kernels read the
// iteration number and every size they need from device memory, so one graph
// serves every later iteration.
static int capture_iterations(st_problem *p, int n, hipGraphExec_t *out) {
    const int64_t B = p->prm.batch;
    const st_samples smp = work_samples(p);
    if (!p->cap_stream) ST_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = p->cap_stream;
    ST_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = ST_OK;
    for (int i = 0; i < n && rc == ST_OK; ++i) {
        rc = sample_batch(p, -1, B, smp, cs, true);
        if (rc == ST_OK) rc = extend_batch(p, B, smp, nullptr, cs, true);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != ST_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return ST_EHIP;
    }
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        set_error("graph instantiation failed: %s", hipGetErrorString(e2));
        return ST_EHIP;
    }
    // the graph's device-side set-up now, not in its first replay
    ST_HIP(hipGraphUpload(*out, cs));
    ST_HIP(hipStreamSynchronize(cs));
    return ST_OK;
}

constexpr int kGraphChunk = 4;

// Launch set-up of the planner's iterations: work and edge buffers for the
// problem's samples per iteration and (graph replays) the graphs of one and of
// kGraphChunk iterations.  Synchronous; a no-op once done.
static int iterate_prepare(st_problem *p) {
    const int64_t B = p->prm.batch;
    int rc = work_reserve(p, B);
    if (rc != ST_OK) return rc;
    if (p->ebufs.cap < B) {
        graphs_free(p);
        if ((rc = edge_bufs_reserve(p->ebufs, B)) != ST_OK) return rc;
    }
    if (p->prof || !p->use_graphs) return ST_OK;
    if (p->graph_B != B || !p->graph[0] || !p->graph[1]) {
        graphs_free(p);
        ST_HIP(hipDeviceSynchronize());
        if ((rc = capture_iterations(p, 1, &p->graph[0])) != ST_OK) return rc;
        if ((rc = capture_iterations(p, kGraphChunk, &p->graph[1])) != ST_OK) return rc;
        p->graph_B = B;
    }
    return ST_OK;
}

static int iterate(st_problem *p, int64_t iters, hipStream_t s) {
    const int64_t B = p->prm.batch;
    int rc = iterate_prepare(p);
    if (rc != ST_OK) return rc;
    if (p->prof || !p->use_graphs) {
        // eager launches (stage timing records events between kernels)
        const st_samples smp = work_samples(p);
        for (int64_t i = 0; i < iters; ++i) {
            if ((rc = sample_batch(p, -1, B, smp, s, true)) != ST_OK) return rc;
            if ((rc = extend_batch(p, B, smp, nullptr, s, true)) != ST_OK) return rc;
            p->iter++;
        }
        return ST_OK;
    }
    int64_t left = iters;
    while (left >= kGraphChunk) {
        ST_HIP(hipGraphLaunch(p->graph[1], s));
        left -= kGraphChunk;
    }
    while (left > 0) {
        ST_HIP(hipGraphLaunch(p->graph[0], s));
        --left;
    }
    p->iter += iters;
    return ST_OK;
}

// Start state check and the trivial case q_s = q_g (arrival at time 0 when
// the arrival range allows it).  Synchronous.
int start_check(st_problem *p, bool *start_free, bool *trivial) {
    const int d = p->d, W = d + 1;
    bool same = true;
    for (int j = 0; j < d; ++j) same = same && p->q_s[j] == p->q_g[j];
    float *dx = nullptr;
    uint8_t *dfree = nullptr;
    ST_HIP(hipMalloc((void **)&dx, W * sizeof(float)));
    ST_HIP(hipMalloc((void **)&dfree, 1));
    std::vector<float> xs(W);
    for (int j = 0; j < d; ++j) xs[j] = (float)p->q_s[j];
    xs[d] = 0.f;
    ST_HIP(hipMemcpy(dx, xs.data(), W * sizeof(float), hipMemcpyHostToDevice));
    ST_HIP(launch_check_states(p->sc, 1, dx, dfree, 0));
    uint8_t f = 0;
    ST_HIP(hipMemcpy(&f, dfree, 1, hipMemcpyDeviceToHost));
    (void)hipFree(dx);
    (void)hipFree(dfree);
    *start_free = f != 0;
    *trivial = same && f && p->L <= 0.0;
    return ST_OK;
}

// The incumbent path (forward chain, then backward chain) into host memory.
// The chain lengths are read first, so the copy is sized exactly.
int fetch_path(st_problem *p, hipStream_t s, st_path *out) {
    const int W = p->d + 1;
    int32_t *dlen = nullptr;
    float *dpath = nullptr;
    PlanDev host;
    int32_t len[2] = {0, 0};
    int rc = ST_OK;
    if (hipMalloc((void **)&dlen, 2 * sizeof(int32_t)) != hipSuccess) {
        set_error("path extraction: out of device memory");
        return ST_ENOMEM;
    }
    k_path_len<<<1, 1, 0, s>>>(p->tree, p->d_plan, dlen);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(len, dlen, sizeof len, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&host, p->d_plan, sizeof(PlanDev), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("path extraction: device copy failed");
        rc = ST_EHIP;
    } else if (len[0] < 0 || len[1] < 0) {
        set_error("path extraction: a parent chain does not end at a root");
        rc = ST_EHIP;
    }
    const int64_t n = (int64_t)len[0] + len[1];
    if (rc == ST_OK && n > 0) {
        if (hipMalloc((void **)&dpath, (size_t)n * W * sizeof(float)) != hipSuccess) {
            set_error("path extraction: out of device memory");
            rc = ST_ENOMEM;
        } else {
            std::vector<float> buf((size_t)n * W);
            k_path_copy<<<1, 1, 0, s>>>(p->tree, p->d_plan, len[0], len[1], dpath);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(buf.data(), dpath, buf.size() * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("path extraction: device copy failed");
                rc = ST_EHIP;
            } else {
                out->n_states = n;
                out->states = (double *)malloc(sizeof(double) * buf.size());
                if (!out->states) {
                    set_error("path extraction: out of host memory");
                    rc = ST_ENOMEM;
                    out->n_states = 0;
                } else {
                    for (size_t i = 0; i < buf.size(); ++i) out->states[i] = buf[i];
                }
            }
        }
    }
    if (rc == ST_OK) {
        out->dof = p->d;
        out->iterations = p->iter;
        out->arrival = host.U;
        out->length = host.C;
        if (host.first_iter >= 0) out->first_solution_iter = host.first_iter;
        if (n == 0) {
            rc = ST_NO_SOLUTION;
            // growth stopped by full pools is reported as a capacity error
            if (host.overflow) {
                set_error("no solution and the tree capacity is exhausted (inserts were dropped)");
                rc = ST_ECAPACITY;
            }
        }
    }
    if (dpath) (void)hipFree(dpath);
    (void)hipFree(dlen);
    return rc;
}

}  // namespace st

using namespace st;

extern "C" {

int st_nearest(st_problem *p, int32_t set, int32_t metric, int32_t sigma, int64_t M, const float *xq,
               int32_t *idx_out, float *dist_out, void *stream) {
    if (!p || M < 0 || (M > 0 && (!xq || !idx_out))) {
        set_error("st_nearest: bad arguments");
        return ST_EINVAL;
    }
    if (metric != ST_METRIC_RHO && metric != ST_METRIC_CONFIG) {
        set_error("st_nearest: unknown metric %d", metric);
        return ST_EINVAL;
    }
    if (sigma != 1 && sigma != -1) {
        set_error("st_nearest: sigma must be +1 or -1");
        return ST_EINVAL;
    }
    if (set != ST_SET_FORWARD && set != ST_SET_ALL_BACKWARD && (set < 0 || set >= p->prm.n_groups)) {
        set_error("st_nearest: unknown set %d", set);
        return ST_EINVAL;
    }
    return nearest_set(p, set, metric, sigma, M, xq, idx_out, dist_out, (hipStream_t)stream);
}

int st_sample_batch(st_problem *p, int64_t iter, int64_t B, const st_samples *out, void *stream) {
    if (!p || !out || B < 0 || (B > 0 && (!out->dir || !out->flags || !out->grp || !out->T || !out->qr || !out->tr))) {
        set_error("st_sample_batch: bad arguments");
        return ST_EINVAL;
    }
    if (B == 0) return ST_OK;
    return sample_batch(p, iter, B, *out, (hipStream_t)stream, false);
}

int st_extend_batch(st_problem *p, int64_t B, const st_samples *s, const st_extend_out *o, void *stream) {
    if (!p || !s || B < 0 || (B > 0 && (!s->dir || !s->flags || !s->grp || !s->T || !s->qr || !s->tr))) {
        set_error("st_extend_batch: bad arguments");
        return ST_EINVAL;
    }
    if (B == 0) return ST_OK;
    int rc = extend_batch(p, B, *s, o, (hipStream_t)stream, false);
    if (rc == ST_OK) p->iter++;
    return rc;
}

int st_proposal_set(st_problem *p, const float *z, float mix, void *stream) {
    if (!p || !(mix >= 0.f && mix <= 1.f)) {
        set_error("st_proposal_set: bad arguments");
        return ST_EINVAL;
    }
    k_prop_set<<<1, 1, 0, (hipStream_t)stream>>>(p->d_plan, z, mix);
    ST_HIP(hipGetLastError());
    return ST_OK;
}

int st_iterate(st_problem *p, int64_t iters, void *stream) {
    if (!p || iters < 0) {
        set_error("st_iterate: bad arguments");
        return ST_EINVAL;
    }
    return iterate(p, iters, (hipStream_t)stream);
}

int st_plan(st_problem *p, const st_budget *b, st_path *out) {
    if (!p || !b || !out) {
        set_error("st_plan: bad arguments");
        return ST_EINVAL;
    }
    memset(out, 0, sizeof *out);
    out->dof = p->d;
    out->first_solution_iter = -1;
    out->arrival = INFINITY;
    out->length = INFINITY;
    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    const int d = p->d, W = d + 1;
    bool start_free = false, trivial = false;
    int rc0 = start_check(p, &start_free, &trivial);
    if (rc0 != ST_OK) return rc0;
    if (trivial) {
        out->n_states = 1;
        out->states = (double *)malloc(sizeof(double) * W);
        for (int j = 0; j < d; ++j) out->states[j] = p->q_s[j];
        out->states[d] = 0.0;
        out->arrival = 0.0;
        out->length = 0.0;
        out->total_ms = ms_since();
        return ST_TRIVIAL;
    }
    if (!start_free) {
        out->total_ms = ms_since();
        return ST_NO_SOLUTION;
    }
    // work the caller queued on other streams (state import, proposal) comes first
    ST_HIP(hipDeviceSynchronize());
    hipStream_t s = nullptr;
    ST_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    PlanDev *host = nullptr;
    ST_HIP(hipHostMalloc((void **)&host, sizeof(PlanDev), hipHostMallocDefault));
    // the launch set-up (buffers, graph capture) before the first solution's
    // clock, which then runs on the device: from an event ahead of the first
    // launch to one behind the launches that found the solution
    int rc = iterate_prepare(p);
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (rc == ST_OK && (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess ||
                        hipEventRecord(ev[0], s) != hipSuccess)) {
        set_error("st_plan: event set-up failed");
        rc = ST_EHIP;
    }
    const int chunk = b->iters_per_sync > 0 ? b->iters_per_sync : 8;
    int64_t done_iters = 0;
    while (rc == ST_OK) {
        int64_t n = chunk;
        if (b->max_iters > 0) n = std::min<int64_t>(n, b->max_iters - done_iters);
        if (n <= 0) break;
        if ((rc = iterate(p, n, s)) != ST_OK) break;
        done_iters += n;
        if (hipEventRecord(ev[1], s) != hipSuccess ||
            hipMemcpyAsync(host, p->d_plan, sizeof(PlanDev), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            set_error("st_plan: device synchronisation failed");
            rc = ST_EHIP;
            break;
        }
        if (host->first_iter >= 0 && out->first_solution_iter < 0) {
            out->first_solution_iter = host->first_iter;
            float t = 0.f;
            if (hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess) {
                set_error("st_plan: event timing failed");
                rc = ST_EHIP;
                break;
            }
            out->first_solution_ms = t;
        }
        if (host->done) break;
        if (b->stop_at_first && host->first_iter >= 0) break;
        if (b->max_ms > 0 && ms_since() >= b->max_ms) break;
        if (b->max_iters <= 0 && b->max_ms <= 0 && !b->stop_at_first) break;
    }
    if (rc == ST_OK) rc = fetch_path(p, s, out);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    (void)hipHostFree(host);
    (void)hipStreamDestroy(s);
    out->total_ms = ms_since();
    return rc;
}

int st_profile_enable(st_problem *p, int32_t enable) {
    if (!p) {
        set_error("st_profile_enable: null problem");
        return ST_EINVAL;
    }
    ST_HIP(hipDeviceSynchronize());
    p->prof = enable != 0;
    p->prof_used = 0;
    return ST_OK;
}

int st_profile_read(st_problem *p, double *ms, int64_t *marks) {
    if (!p || !ms) {
        set_error("st_profile_read: bad arguments");
        return ST_EINVAL;
    }
    ST_HIP(hipDeviceSynchronize());
    for (int i = 0; i < ST_PROFILE_STAGES; ++i) {
        ms[i] = 0.0;
        if (marks) marks[i] = 0;
    }
    // the interval between consecutive marks belongs to the earlier mark's stage
    for (size_t i = 0; i + 1 < p->prof_used; ++i) {
        const int st_ = p->prof_stage[i];
        if (st_ == kStEnd) continue;
        float t = 0.f;
        ST_HIP(hipEventElapsedTime(&t, p->prof_ev[i], p->prof_ev[i + 1]));
        ms[st_] += t;
        if (marks) marks[st_]++;
    }
    p->prof_used = 0;
    return ST_OK;
}

int st_work_counters(st_problem *p, uint64_t *out) {
    if (!p || !out) {
        set_error("st_work_counters: bad arguments");
        return ST_EINVAL;
    }
    ST_HIP(hipDeviceSynchronize());
    PlanDev pl;
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out[i] = pl.work[i];
    return ST_OK;
}

void st_path_free(st_path *path) {
    if (!path) return;
    free(path->states);
    path->states = nullptr;
    path->n_states = 0;
}

}  // extern "C"
