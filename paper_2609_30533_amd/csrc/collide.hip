// collide.hip -- state and edge validity kernels (Sec. IV-B: edges are checked
// along their interpolation; Sec. VI: obstacles at the absolute query time).
//
// One space-time state per lane; after each robot link the wave ballots its
// hits so that lanes above a known hit of their group stop early.
#include <type_traits>

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

constexpr int32_t kNoHit = 0x7fffffff;

__global__ __launch_bounds__(256) void k_edge_plan(int64_t E, int d, double v, double h, int L, int mmax,
                                                   const float *__restrict__ xa, const float *__restrict__ xb,
                                                   const uint8_t *__restrict__ valid, EdgeBufs eb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int w = d + 1;
    int m = 0;
    if (e < E && !(valid && !valid[e])) {
        const float *A = xa + e * w, *B = xb + e * w;
        if (A[d] > B[d]) { const float *tmp = A; A = B; B = tmp; }
        double D2 = 0.0;
        for (int j = 0; j < d; ++j) {
            const double dq = (double)B[j] - (double)A[j];
            D2 += dq * dq;
        }
        const double span = fmax(sqrt(D2), v * ((double)B[d] - (double)A[d]));
        int64_t n = (int64_t)ceil(span / h);
        if (n < 1) n = 1;
        if (n > (1ll << 30)) n = 1ll << 30;
        const int64_t c = (n + L) / L;
        m = (int)(c < mmax ? c : mmax);
        eb.n[e] = (int32_t)n;
        eb.hit[e] = kNoHit;
    } else if (e < E) {
        eb.n[e] = -1;
    }
    for (int r = 0; r < mmax; ++r) {
        const bool want = m > r;
        const uint64_t mask = __ballot(want);
        if (mask == 0) break;
        const int leader = __builtin_ctzll(mask);
        int base = 0;
        if (lane == leader) base = atomicAdd(&eb.cnt[r], __popcll(mask));
        base = __shfl(base, leader, 64);
        if (want) {
            const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
            eb.items[(int64_t)r * eb.cap + slot] = make_int2((int)e, r);
        }
    }
}

template <int KIND, int OT, int OBS>
__global__ __launch_bounds__(256) void k_edge_items(SceneDev sc, const float *__restrict__ xa,
                                                    const float *__restrict__ xb, EdgeBufs eb, int lpe_shift) {
    extern __shared__ float4 lds[];
    stage_obstacles(sc, lds);
    int32_t pre[17];
    pre[0] = 0;
    for (int r = 0; r < eb.mmax; ++r) pre[r + 1] = pre[r] + eb.cnt[r];
    const int64_t total = pre[eb.mmax];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpe = 1 << lpe_shift;
    const int G = 64 >> lpe_shift;
    const int sub = lane & (lpe - 1), gsel = lane >> lpe_shift;
    const uint64_t gbits = lpe == 64 ? ~0ull : ((1ull << lpe) - 1ull);
    const uint64_t group_mask = gbits << (gsel * lpe);
    const uint64_t lower_mask = group_mask & ((1ull << lane) - 1ull);
    const int w = sc.d + 1;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6) * G;
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * G; base < total; base += stride) {
        const int64_t v = base + gsel;
        bool done = !(v < total);
        int e = 0, rank = 0;
        if (!done) {
            int r = 0;
            while (v >= pre[r + 1]) ++r;
            const int2 it = eb.items[(int64_t)r * eb.cap + (v - pre[r])];
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
            c_e = (n + lpe) / lpe;
            m = c_e < eb.mmax ? c_e : eb.mmax;
        }
        const float inv_n = 1.0f / (float)n;
        for (int64_t c = rank;; c += m) {
            if (!done) {
                if (c >= c_e) done = true;
                else if (__atomic_load_n(&eb.hit[e], __ATOMIC_RELAXED) < c * lpe) done = true;
            }
            const int64_t j = c * lpe + sub;
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
            const bool hit = state_hits<KIND, OT, OBS, true>(sc, lds, q, t, act, group_mask, lower_mask);
            const uint64_t hm = __ballot(hit && act) & group_mask;
            if (!done && hm) {
                atomicMin(&eb.hit[e], (int32_t)(c * lpe + (__builtin_ctzll(hm) - gsel * lpe)));
                done = true;
            }
            if (__ballot(!done) == 0) break;
        }
    }
}

__global__ __launch_bounds__(256) void k_edge_finish(int64_t E, const uint8_t *__restrict__ valid, EdgeBufs eb,
                                                     uint8_t *__restrict__ free_out, int32_t *__restrict__ fh_out,
                                                     unsigned long long *__restrict__ work) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    unsigned long long states = 0, edges = 0;
    if (e < E && !(valid && !valid[e])) {
        const int32_t h = eb.hit[e];
        const bool fr = h == kNoHit;
        free_out[e] = fr ? 1 : 0;
        if (fh_out) fh_out[e] = fr ? -1 : h;
        // algorithmic work: the states up to the first hit, all n+1 when free
        states = fr ? (unsigned long long)eb.n[e] + 1ull : (unsigned long long)h + 1ull;
        edges = 1;
    }
    if (work) {
        for (int o = 32; o > 0; o >>= 1) {
            states += __shfl_down(states, o, 64);
            edges += __shfl_down(edges, o, 64);
        }
        if (lane == 0 && edges) {
            atomicAdd(&work[0], edges);
            atomicAdd(&work[1], states);
        }
    }
    // the rank lists are consumed: leave them empty for the next launch
    if (blockIdx.x == 0 && threadIdx.x < eb.mmax) eb.cnt[threadIdx.x] = 0;
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

// Calls f(IC<KIND>, IC<OT>, IC<OBS>) for the scene's robot kind, obstacle tile
// and obstacle-time mode.
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
    else by_obs(IC<kDH>{});
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
    ST_HIP(hipMalloc((void **)&eb.cnt, 16 * sizeof(int32_t)));
    ST_HIP(hipMemset(eb.cnt, 0, 16 * sizeof(int32_t)));
    return ST_OK;
}

void edge_bufs_free(EdgeBufs &eb) {
    void *b[] = {eb.n, eb.hit, eb.items, eb.cnt};
    for (void *x : b)
        if (x) (void)hipFree(x);
    eb = EdgeBufs{};
}

hipError_t launch_check_edges(const SceneDev &sc, const EdgeBufs &eb, int64_t E, const float *xa, const float *xb,
                              const uint8_t *valid, uint8_t *free_out, int32_t *first_hit, int lpe_shift,
                              hipStream_t s, unsigned long long *work) {
    if (E <= 0) return hipSuccess;
    if (E > eb.cap) return hipErrorInvalidValue;
    const int L = 1 << lpe_shift;
    const int eblocks = (int)((E + 255) / 256);
    k_edge_plan<<<eblocks, 256, 0, s>>>(E, sc.d, sc.v_d, sc.h_d, L, eb.mmax, xa, xb, valid, eb);
    // enough groups to cover the first-rank items of every edge, capped so
    // that a grid-stride loop covers the rest
    const int G = 64 >> lpe_shift;
    const int64_t per_block = 4 * (int64_t)G;
    const int64_t want = (E + per_block - 1) / per_block;
    const int blocks = (int)(want < 8192 ? (want < 1024 ? 1024 : want) : 8192);
    const size_t lds = scene_lds_bytes(sc);
    dispatch_scene(sc, [&](auto kind, auto ot, auto obs) {
        k_edge_items<decltype(kind)::value, decltype(ot)::value, decltype(obs)::value>
            <<<dim3(blocks), dim3(256), lds, s>>>(sc, xa, xb, eb, lpe_shift);
    });
    k_edge_finish<<<eblocks, 256, 0, s>>>(E, valid, eb, free_out, first_hit, work);
    return hipGetLastError();
}

}  // namespace st
