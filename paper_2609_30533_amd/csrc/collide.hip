// collide.hip -- state and edge validity kernels (Sec. IV-B: edges are checked
// along their interpolation; Sec. VI: obstacles at the absolute query time).
//
// One space-time state per lane; after each robot link the wave ballots its
// hits so that lanes above a known hit of their group stop early.
#include <algorithm>
#include <type_traits>

#include "edge_flat.hpp"
#include "st_internal.hpp"

namespace st {

template <int KIND, int OT, int OBS>
__global__ __launch_bounds__(256) void k_check_states(SceneDev sc, int64_t M, const float *__restrict__ x,
                                                      uint8_t *__restrict__ free_out) {
    extern __shared__ float4 lds[];
    stage_obstacles(sc, lds);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int w = sc.d + 1;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < M; base += stride) {
        const int64_t i = base + lane;
        const bool act = i < M;
        float q[kMaxDof];
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j) q[j] = (act && j < sc.d) ? x[i * w + j] : 0.f;
        if (act) t = x[i * w + sc.d];
        const uint64_t self = 1ull << lane;
        const bool hit = state_hits<KIND, OT, OBS, true>(sc, lds, q, t, act, self, 0ull);
        if (act) free_out[i] = hit ? 0 : 1;
    }
}

// ---------------------------------------------------------------------------
// Exact continuous edge check for a translating robot: the edge's time span
// is cut where an obstacle changes segment; on each piece the robot (linear
// along the edge) and the obstacle (one constant-velocity segment, or held)
// move linearly, so a sphere pair's relative position is affine in time and
// its closest approach is u* = clamp(-p0.(p1 - p0) / |p1 - p0|^2, 0, 1)
// between the piece's end values.  The box and horizon hold along the edge
// iff they hold at both endpoints (convex sets).  One thread per edge.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void obstacle_at(const float4 *lds, int n_seg, int o, int k, float t, float &x, float &y,
                                            float &z) {
    float nx, ny, nz;
    obstacle_n(lds, n_seg, o, k, t, nx, ny, nz);
    x = -0.5f * nx;
    y = -0.5f * ny;
    z = -0.5f * nz;
}

__global__ __launch_bounds__(256) void k_edge_continuous(SceneDev sc, int64_t E, const float *__restrict__ xa,
                                                         const float *__restrict__ xb, uint8_t *__restrict__ free_out,
                                                         float *__restrict__ dmin_out) {
    extern __shared__ float4 lds[];
    stage_obstacles(sc, lds);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int d = sc.d, W = d + 1;
    const float *A = xa + e * W, *B = xb + e * W;
    if (A[d] > B[d]) { const float *tmp = A; A = B; B = tmp; }
    float qa[3] = {0.f, 0.f, 0.f}, qb[3] = {0.f, 0.f, 0.f};
    for (int j = 0; j < d && j < 3; ++j) {
        qa[j] = A[j];
        qb[j] = B[j];
    }
    bool ok = true;
    for (int j = 0; j < d; ++j)
        ok = ok && A[j] >= sc.q_lo[j] && A[j] <= sc.q_hi[j] && B[j] >= sc.q_lo[j] && B[j] <= sc.q_hi[j];
    const float ta = A[d], tb = B[d], T = tb - ta;
    ok = ok && ta >= 0.f && tb <= sc.H;
    float best = INFINITY;
    const float *lt = reinterpret_cast<const float *>(lds + sc.lds_t);
    for (int o = 0; o < sc.O; ++o) {
        const int ka = sc.obs_mode == kObsShared ? shared_segment(sc, ta) : generic_segment(sc, lds, o, ta);
        const int kb = sc.obs_mode == kObsShared ? shared_segment(sc, tb) : generic_segment(sc, lds, o, tb);
        for (int k = ka; k <= kb; ++k) {
            const float tk1 = sc.obs_mode == kObsShared ? sc.seg_t[k + 1] : lt[o * (sc.n_seg + 1) + k + 1];
            const float t0 = k == ka ? ta : lds[(o * sc.n_seg + k) * 2].w;
            const float t1 = k == kb ? tb : tk1;
            float c0x, c0y, c0z, c1x, c1y, c1z;
            obstacle_at(lds, sc.n_seg, o, k, t0, c0x, c0y, c0z);
            obstacle_at(lds, sc.n_seg, o, k, t1, c1x, c1y, c1z);
            const float f0 = T > 0.f ? (t0 - ta) / T : 0.f, f1 = T > 0.f ? (t1 - ta) / T : 0.f;
            float r0[3], r1[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r0[c] = fmaf(f0, qb[c] - qa[c], qa[c]);
                r1[c] = fmaf(f1, qb[c] - qa[c], qa[c]);
            }
            for (int s = 0; s < sc.S; ++s) {
                const float4 sp = lds[sc.lds_sph + s];
                const float p0x = r0[0] + sp.x - c0x, p0y = r0[1] + sp.y - c0y, p0z = r0[2] + sp.z - c0z;
                const float dx = (r1[0] + sp.x - c1x) - p0x, dy = (r1[1] + sp.y - c1y) - p0y,
                            dz = (r1[2] + sp.z - c1z) - p0z;
                const float pp = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                const float pd = fmaf(p0x, dx, fmaf(p0y, dy, p0z * dz));
                const float u = pp > 0.f ? fminf(fmaxf(-pd / pp, 0.f), 1.f) : 0.f;
                const float mx = fmaf(u, dx, p0x), my = fmaf(u, dy, p0y), mz = fmaf(u, dz, p0z);
                const float dist = sqrtf(fmaf(mx, mx, fmaf(my, my, mz * mz))) - (sp.w + sc.obs_r[o]);
                best = fminf(best, dist);
            }
        }
    }
    free_out[e] = ok && best >= 0.f ? 1 : 0;
    if (dmin_out) dmin_out[e] = best;
}

hipError_t launch_check_edges_continuous(const SceneDev &sc, int64_t E, const float *xa, const float *xb,
                                         uint8_t *free_out, float *dmin_out, hipStream_t s) {
    if (E <= 0) return hipSuccess;
    k_edge_continuous<<<(int)((E + 255) / 256), 256, scene_lds_bytes(sc), s>>>(sc, E, xa, xb, free_out, dmin_out);
    return hipGetLastError();
}

// World centres of the robot's spheres at q_g (one thread per sphere, the
// same kinematics code as the state tests, so the goal-state tests decide
// exactly as a state test at q = q_g would).
__global__ void k_goal_centers(SceneDev sc, float4 *out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= sc.S) return;
    float q[kMaxDof];
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j) q[j] = sc.q_g[j];
    float cx, cy, cz, as;
    if (sc.kind == kTranslate) {
        sphere_translate(sc, q, sc.sph[s], cx, cy, cz, as);
    } else {
        Frame f;
        frame_identity(f);
        for (int l = 1; l <= sc.d && sc.link_first[l] <= s; ++l) dh_compose(sc, l - 1, q[l - 1], f);
        sphere_world(f, sc.sph[s], cx, cy, cz, as);
    }
    out[s] = make_float4(cx, cy, cz, as);
}

hipError_t launch_goal_centers(const SceneDev &sc, float4 *out) {
    if (sc.S <= 0) return hipSuccess;
    k_goal_centers<<<(sc.S + 63) / 64, 64>>>(sc, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Edge checks as a three-kernel pipeline.
//
//   plan    one thread per edge: endpoints ordered by time, the state count
//           n = max(1, ceil(max(D, v dt) / h)) in double precision, the number
//           of L-state chunks c = ceil((n+1)/L), and m = min(c, mmax) work
//           items (e, r), r < m, appended to list r (wave-aggregated atomics);
//   items   a group of L lanes takes one item and walks the chunks r, r+m,
//           r+2m, ... of its edge; lane j checks state c L + j.  Lists are
//           processed in rank order, so first chunks of all edges run first;
//           a group skips a chunk once a hit below the chunk is known, and a
//           hit is merged into the edge with atomicMin (the least colliding
//           index wins, independent of the item schedule);
//   finish  free / first hit per edge and the work counters.
// Long edges are thus spread over up to mmax groups instead of serialising in
// one wave.
// ---------------------------------------------------------------------------

constexpr int kMaxItems = 16;   // work items per edge at most

__device__ __forceinline__ void edge_plan_body(const EdgeArgs &a, int bx) {
    const EdgeBufs &eb = a.eb;
    // states per chunk: lanes per chunk over lanes per state
    const int d = a.sc.d, L = 1 << (a.lpe_shift - a.split_shift), mmax = eb.mmax;
    const double v = a.sc.v_d, h = a.sc.h_d;
    const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int m = 0;
    if (e < a.E) {
        // the flag and both rows in flight together
        float A[kMaxDof + 1], B[kMaxDof + 1];
        load_edge_rows(a.xa, a.xb, e, d, A, B);
        const bool vld = !a.valid || a.valid[e];
        if (vld) {
            const int64_t n = edge_states(A, B, d, v, h);
            const int64_t c = (n + L) / L;
            m = (int)(c < mmax ? c : mmax);
            eb.n[e] = (int32_t)n;
            eb.hit[e] = kNoHit;
        } else {
            eb.n[e] = -1;
        }
    }
    // rank lists: positions within the block from LDS counters (one per wave
    // and rank), then one global atomic per rank and block; every rank's
    // global counter sits on its own cache line
    __shared__ int wcnt[4][kMaxItems], bbase[kMaxItems];
    const int wave = threadIdx.x >> 6;
    uint64_t masks[kMaxItems];
#pragma unroll
    for (int r = 0; r < kMaxItems; ++r) {
        masks[r] = r < mmax ? __ballot(m > r) : 0ull;
        if (lane == 0) wcnt[wave][r] = __popcll(masks[r]);
    }
    __syncthreads();
    if (threadIdx.x < mmax) {
        const int r = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            const int c = wcnt[w][r];
            wcnt[w][r] = tot;
            tot += c;
        }
        bbase[r] = tot > 0 ? atomicAdd(&eb.cnt[r * kCntStride], tot) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kMaxItems; ++r) {
        if (m > r) {
            const int slot = bbase[r] + wcnt[wave][r] + __popcll(masks[r] & ((1ull << lane) - 1ull));
            eb.items[(int64_t)r * eb.cap + slot] = make_int2((int)e, r);
        }
    }
}

template <int KIND, int OT, int OBS, int SPLIT>
__device__ __forceinline__ void edge_items_body(const EdgeArgs &a, float4 *lds, int bx, int nbx) {
    const SceneDev &sc = a.sc;
    const EdgeBufs &eb = a.eb;
    const float *__restrict__ xa = a.xa;
    const float *__restrict__ xb = a.xb;
    // prefix of the rank lists' lengths: the kMaxItems counters are read
    // together (a loop up to mmax would wait for each load in turn); the
    // prefix goes to LDS (written here, visible after the staging barrier),
    // where a lane's lookup by its own rank is a plain LDS read
    __shared__ int32_t s_pre[kMaxItems + 1];
    int32_t cr[kMaxItems];
#pragma unroll
    for (int r = 0; r < kMaxItems; ++r) cr[r] = eb.cnt[r * kCntStride];
    int32_t total32 = 0, mine = 0;
#pragma unroll
    for (int r = 0; r < kMaxItems; ++r) {
        if ((int)threadIdx.x == r) mine = total32;
        total32 += r < eb.mmax ? cr[r] : 0;
    }
    if (threadIdx.x == kMaxItems) mine = total32;
    const int64_t total = total32;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpe_shift = a.lpe_shift;
    const int lpe = 1 << lpe_shift;
    const int G = 64 >> lpe_shift;
    // a block without any item leaves before staging the scene (the grid is
    // sized for the largest launch; the item count is known only here)
    if ((int64_t)bx * (blockDim.x >> 6) * G >= total) return;
    if (threadIdx.x <= kMaxItems) s_pre[threadIdx.x] = mine;
    stage_obstacles(sc, lds);
    const int sub = lane & (lpe - 1), gsel = lane >> lpe_shift;
    // SPLIT lanes per state: states per chunk ls, the lane's state slot and part
    const int ls = lpe / SPLIT, slot = sub / SPLIT, part = sub & (SPLIT - 1);
    const uint64_t gbits = lpe == 64 ? ~0ull : ((1ull << lpe) - 1ull);
    const uint64_t group_mask = gbits << (gsel * lpe);
    const uint64_t lower_mask = group_mask & ((1ull << (lane & ~(SPLIT - 1))) - 1ull);
    const int w = sc.d + 1;
    const int64_t stride = (int64_t)nbx * (blockDim.x >> 6) * G;
    for (int64_t base = ((int64_t)bx * (blockDim.x >> 6) + wave) * G; base < total; base += stride) {
        const int64_t v = base + gsel;
        bool done = !(v < total);
        int e = 0, rank = 0;
        if (!done) {
            int r = 0;
            while (v >= s_pre[r + 1]) ++r;
            const int2 it = eb.items[(int64_t)r * eb.cap + (v - s_pre[r])];
            e = it.x;
            rank = it.y;
        }
        const float *A = xa, *B = xb;
        int64_t n = 1, c_e = 0, m = 1;
        if (!done) {
            A = xa + (int64_t)e * w;
            B = xb + (int64_t)e * w;
            if (A[sc.d] > B[sc.d]) { const float *tmp = A; A = B; B = tmp; }
            n = eb.n[e];
            c_e = (n + ls) / ls;
            m = c_e < eb.mmax ? c_e : eb.mmax;
        }
        const float inv_n = 1.0f / (float)n;
        for (int64_t c = rank;; c += m) {
            if (!done) {
                if (c >= c_e) done = true;
                else if (__atomic_load_n(&eb.hit[e], __ATOMIC_RELAXED) < c * ls) done = true;
            }
            const int64_t j = c * ls + slot;
            const bool act = !done && j <= n;
            float q[kMaxDof];
            float t = 0.f;
            if (act && j == n) {
                // the last state is the endpoint itself
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) q[k] = k < sc.d ? B[k] : 0.f;
                t = B[sc.d];
            } else if (act) {
                const float s = (float)j * inv_n;
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) q[k] = k < sc.d ? fmaf(s, B[k] - A[k], A[k]) : 0.f;
                t = fmaf(s, B[sc.d] - A[sc.d], A[sc.d]);
            } else {
#pragma unroll
                for (int k = 0; k < kMaxDof; ++k) q[k] = 0.f;
            }
            const bool hit = state_hits<KIND, OT, OBS, true, SPLIT>(sc, lds, q, t, act, group_mask, lower_mask, part);
            const uint64_t hm = __ballot(hit && act) & group_mask;
            if (!done && hm) {
                // one atomic per group: its lowest hitting lane
                if (lane == __builtin_ctzll(hm))
                    atomicMin(&eb.hit[e], (int32_t)(c * ls + ((__builtin_ctzll(hm) - gsel * lpe) / SPLIT)));
                done = true;
            }
            if (__ballot(!done) == 0) break;
        }
    }
}

__device__ __forceinline__ void edge_finish_body(const EdgeArgs &a, int bx) {
    const EdgeBufs &eb = a.eb;
    const int64_t e = (int64_t)bx * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    unsigned long long states = 0, edges = 0;
    if (e < a.E && !(a.valid && !a.valid[e])) {
        const int32_t h = eb.hit[e];
        const bool fr = h == kNoHit;
        a.free_out[e] = fr ? 1 : 0;
        if (a.first_hit) a.first_hit[e] = fr ? -1 : h;
        // algorithmic work: the states up to the first hit, all n+1 when free
        states = fr ? (unsigned long long)eb.n[e] + 1ull : (unsigned long long)h + 1ull;
        edges = 1;
    }
    if (a.work) {
        for (int o = 32; o > 0; o >>= 1) {
            states += __shfl_down(states, o, 64);
            edges += __shfl_down(edges, o, 64);
        }
        if (lane == 0 && edges) {
            atomicAdd(&a.work[0], edges);
            atomicAdd(&a.work[1], states);
        }
    }
    // the rank lists are consumed: leave them empty for the next launch
    if (bx == 0 && threadIdx.x < eb.mmax) eb.cnt[threadIdx.x * kCntStride] = 0;
}

__global__ __launch_bounds__(256) void k_edge_plan(EdgeArgs a) { edge_plan_body(a, blockIdx.x); }

template <int KIND, int OT, int OBS, int SPLIT>
__global__ __launch_bounds__(256) void k_edge_items(EdgeArgs a) {
    extern __shared__ float4 lds[];
    edge_items_body<KIND, OT, OBS, SPLIT>(a, lds, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void k_edge_finish(EdgeArgs a) { edge_finish_body(a, blockIdx.x); }

// Many problems per launch: blockIdx.y selects the problem's record; the
// per-scene-class item kernel takes its member from blockIdx.x (through
// `members`; members vary fastest, so every member's first blocks, the ones
// that hold its items, are dispatched before the members' empty blocks).
// Blocks past the problem's own grid leave at once.
__global__ __launch_bounds__(256) void k_edge_plan_multi(const EdgeArgs *__restrict__ av) {
    const EdgeArgs &a = av[blockIdx.y];
    if ((int)blockIdx.x >= a.nb_edge) return;
    edge_plan_body(a, blockIdx.x);
}

template <int KIND, int OT, int OBS, int SPLIT>
__global__ __launch_bounds__(256) void k_edge_items_multi(const EdgeArgs *__restrict__ av,
                                                          const int32_t *__restrict__ members) {
    extern __shared__ float4 lds[];
    const EdgeArgs &a = av[members[blockIdx.x]];
    if ((int)blockIdx.y >= a.nb_items) return;
    edge_items_body<KIND, OT, OBS, SPLIT>(a, lds, blockIdx.y, a.nb_items);
}

__global__ __launch_bounds__(256) void k_edge_finish_multi(const EdgeArgs *__restrict__ av) {
    const EdgeArgs &a = av[blockIdx.y];
    if ((int)blockIdx.x >= a.nb_edge) return;
    edge_finish_body(a, blockIdx.x);
}

// Obstacles held in registers per tile: 4, 8 or 16 (more obstacles run as
// several tiles; 32 would cost occupancy for little gain).
static int ot_for(int O_pad) {
    if (O_pad <= 4) return 4;
    if (O_pad <= 8) return 8;
    return 16;
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<KIND>, IC<OT>, IC<OBS>) for the scene's robot kind (an arm with
// static geometry as kDHStatic), obstacle tile and obstacle-time mode.
template <class F>
static void dispatch_scene(const SceneDev &sc, F &&f) {
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
    else if (sc.stat) by_obs(IC<kDHStatic>{});
    else by_obs(IC<kDH>{});
}

// f(IC<KIND>, IC<OT>, IC<OBS>, IC<SPLIT>): the lane split of a state applies
// to the arm kind only (a translating robot has too few spheres to share).
template <class F>
static void dispatch_split(const SceneDev &sc, int split_shift, F &&f) {
    dispatch_scene(sc, [&](auto kind, auto ot, auto obs) {
        if (decltype(kind)::value == kTranslate) {
            f(kind, ot, obs, IC<1>{});
        } else {
            switch (split_shift) {
                case 1: f(kind, ot, obs, IC<2>{}); break;
                case 2: f(kind, ot, obs, IC<4>{}); break;
                default: f(kind, ot, obs, IC<1>{}); break;
            }
        }
    });
}

size_t scene_lds_bytes(const SceneDev &sc) { return (size_t)sc.lds_f4 * sizeof(float4); }

hipError_t launch_check_states(const SceneDev &sc, int64_t M, const float *x, uint8_t *free_out, hipStream_t s) {
    if (M <= 0) return hipSuccess;
    const int64_t want = (M + 255) / 256;
    const int blocks = (int)(want < 8192 ? want : 8192);
    const size_t lds = scene_lds_bytes(sc);
    dispatch_scene(sc, [&](auto kind, auto ot, auto obs) {
        k_check_states<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value>
            <<<dim3(blocks), dim3(256), lds, s>>>(sc, M, x, free_out);
    });
    return hipGetLastError();
}

int edge_bufs_reserve(EdgeBufs &eb, int64_t E) {
    if (eb.cap >= E && eb.n) return ST_OK;
    if (eb.n) {
        ST_HIP(hipDeviceSynchronize());
        (void)hipFree(eb.n);
        (void)hipFree(eb.hit);
        (void)hipFree(eb.items);
        (void)hipFree(eb.cnt);
    }
    const int64_t cap = E < 4096 ? 4096 : E;
    eb.cap = cap;
    eb.mmax = cap <= (1 << 16) ? 16 : 4;
    ST_HIP(hipMalloc((void **)&eb.n, cap * sizeof(int32_t)));
    ST_HIP(hipMalloc((void **)&eb.hit, cap * sizeof(int32_t)));
    ST_HIP(hipMalloc((void **)&eb.items, (size_t)cap * eb.mmax * sizeof(int2)));
    ST_HIP(hipMalloc((void **)&eb.cnt, kMaxItems * kCntStride * sizeof(int32_t)));
    ST_HIP(hipMemset(eb.cnt, 0, kMaxItems * kCntStride * sizeof(int32_t)));
    return ST_OK;
}

void edge_bufs_free(EdgeBufs &eb) {
    void *b[] = {eb.n, eb.hit, eb.items, eb.cnt};
    for (void *x : b)
        if (x) (void)hipFree(x);
    eb = EdgeBufs{};
}

EdgeArgs edge_args(const SceneDev &sc, const EdgeBufs &eb, int64_t E, const float *xa, const float *xb,
                   const uint8_t *valid, uint8_t *free_out, int32_t *first_hit, int lpe_shift,
                   unsigned long long *work, int min_item_blocks, int split_shift) {
    EdgeArgs a;
    // a translating robot checks one state per lane; a split never exceeds the chunk
    a.split_shift = sc.kind == kTranslate ? 0 : std::max(0, std::min(std::min(split_shift, 2), lpe_shift));
    a.sc = sc;
    a.eb = eb;
    a.xa = xa;
    a.xb = xb;
    a.valid = valid;
    a.free_out = free_out;
    a.first_hit = first_hit;
    a.work = work;
    a.E = E;
    a.lpe_shift = lpe_shift;
    a.nb_edge = (int)((E + 255) / 256);
    // enough groups to cover the first-rank items of every edge, capped so
    // that a grid-stride loop covers the rest
    const int64_t per_block = 4 * (int64_t)(64 >> lpe_shift);
    const int64_t want = (E + per_block - 1) / per_block;
    a.nb_items = (int)std::min<int64_t>(std::max<int64_t>(want, min_item_blocks), 8192);
    a.flat = 0;
    a.skip_finish = 0;
    return a;
}


hipError_t launch_check_edges(const SceneDev &sc, const EdgeBufs &eb, int64_t E, const float *xa, const float *xb,
                              const uint8_t *valid, uint8_t *free_out, int32_t *first_hit, int lpe_shift,
                              hipStream_t s, unsigned long long *work, int split_shift) {
    if (E <= 0) return hipSuccess;
    if (E > eb.cap) return hipErrorInvalidValue;
    return launch_edge_args(edge_args(sc, eb, E, xa, xb, valid, free_out, first_hit, lpe_shift, work, 1024,
                                      split_shift), s);
}

hipError_t launch_edge_args(const EdgeArgs &a, hipStream_t s) {
    if (a.E <= 0) return hipSuccess;
    // the flattened path of extension edges is launched with the steering
    // that produces them (extend.hip)
    if (a.flat) return hipErrorInvalidValue;
    if (a.E > a.eb.cap) return hipErrorInvalidValue;
    k_edge_plan<<<a.nb_edge, 256, 0, s>>>(a);
    const size_t lds = scene_lds_bytes(a.sc);
    dispatch_split(a.sc, a.split_shift, [&](auto kind, auto ot, auto obs, auto split) {
        k_edge_items<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, decltype(split)::value>
            <<<dim3(a.nb_items), dim3(256), lds, s>>>(a);
    });
    if (!a.skip_finish) k_edge_finish<<<a.nb_edge, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_edge_items(const EdgeArgs &a, hipStream_t s) {
    if (a.E <= 0) return hipSuccess;
    if (a.E > a.eb.cap) return hipErrorInvalidValue;
    const size_t lds = scene_lds_bytes(a.sc);
    dispatch_split(a.sc, a.split_shift, [&](auto kind, auto ot, auto obs, auto split) {
        k_edge_items<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, decltype(split)::value>
            <<<dim3(a.nb_items), dim3(256), lds, s>>>(a);
    });
    return hipGetLastError();
}

hipError_t launch_edge_plan_multi(const EdgeArgs *d_args, int P, int max_nb_edge, hipStream_t s) {
    k_edge_plan_multi<<<dim3(max_nb_edge, P), 256, 0, s>>>(d_args);
    return hipGetLastError();
}

hipError_t launch_edge_items_multi(const SceneDev &cls, int split_shift, const EdgeArgs *d_args,
                                   const int32_t *d_members, int n_members, int max_nb_items, size_t lds,
                                   hipStream_t s) {
    dispatch_split(cls, split_shift, [&](auto kind, auto ot, auto obs, auto split) {
        k_edge_items_multi<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value, decltype(split)::value>
            <<<dim3(n_members, max_nb_items), dim3(256), lds, s>>>(d_args, d_members);
    });
    return hipGetLastError();
}

hipError_t launch_edge_finish_multi(const EdgeArgs *d_args, int P, int max_nb_edge, hipStream_t s) {
    k_edge_finish_multi<<<dim3(max_nb_edge, P), 256, 0, s>>>(d_args);
    return hipGetLastError();
}

}  // namespace st
