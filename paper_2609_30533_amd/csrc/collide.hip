// collide.hip -- state and edge validity kernels (Sec. IV-B: edges are checked
// along their interpolation; Sec. VI: obstacles at the absolute query time).
//
// Edge kernel work map: a wave is split into groups of LPE = 64 >> G lanes,
// one edge per group; the group walks the edge's n+1 states in chunks of LPE
// consecutive states (lane j of the group takes state c0 + j).  After each
// robot link the wave ballots its hits, so a group stops as soon as the first
// colliding state of the edge is known (or, without first-hit output, as soon
// as any state collides).
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

template <int KIND, int OT, int OBS, bool FIRST>
__global__ __launch_bounds__(256) void k_check_edges(SceneDev sc, int64_t E, const float *__restrict__ xa,
                                                     const float *__restrict__ xb, const uint8_t *__restrict__ valid,
                                                     uint8_t *__restrict__ free_out, int32_t *__restrict__ fh_out,
                                                     int lpe_shift, unsigned long long *__restrict__ work) {
    extern __shared__ float4 lds[];
    stage_obstacles(sc, lds);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lpe = 1 << lpe_shift;
    const int G = 64 >> lpe_shift;
    const int sub = lane & (lpe - 1), gsel = lane >> lpe_shift;
    const uint64_t gbits = lpe == 64 ? ~0ull : ((1ull << lpe) - 1ull);
    const uint64_t group_mask = gbits << (gsel * lpe);
    const uint64_t lower_mask = group_mask & ((1ull << lane) - 1ull);
    const int w = sc.d + 1;
    const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6) * G;
    for (int64_t base = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * G; base < E; base += stride) {
        const int64_t e = base + gsel;
        bool done = !(e < E) || (valid && !valid[e]);
        float qa[kMaxDof], dq[kMaxDof], qb[kMaxDof];
        float ta = 0.f, dtt = 0.f, tb = 0.f;
        int64_t n = 1;
        if (!done) {
            const float *A = xa + e * w, *B = xb + e * w;
            if (A[sc.d] > B[sc.d]) { const float *tmp = A; A = B; B = tmp; }
            // the state count is taken in double precision so that it agrees
            // with an FP64 evaluation of the same endpoints
            double D2 = 0.0;
#pragma unroll
            for (int j = 0; j < kMaxDof; ++j) {
                if (j < sc.d) {
                    qa[j] = A[j];
                    qb[j] = B[j];
                    dq[j] = B[j] - A[j];
                    const double e = (double)B[j] - (double)A[j];
                    D2 += e * e;
                } else {
                    qa[j] = qb[j] = dq[j] = 0.f;
                }
            }
            ta = A[sc.d];
            tb = B[sc.d];
            dtt = tb - ta;
            const double span = fmax(sqrt(D2), sc.v_d * ((double)tb - (double)ta));
            n = (int64_t)ceil(span / sc.h_d);
            if (n < 1) n = 1;
        }
        const float inv_n = 1.0f / (float)n;
        int32_t hit_at = -1;
        for (int64_t c0 = 0;; c0 += lpe) {
            const int64_t j = c0 + sub;
            const bool act = !done && j <= n;
            float q[kMaxDof];
            float t = 0.f;
            if (act && j == n) {
                // the last state is the endpoint itself
#pragma unroll
                for (int c = 0; c < kMaxDof; ++c) q[c] = qb[c];
                t = tb;
            } else if (act) {
                const float s = (float)j * inv_n;
#pragma unroll
                for (int c = 0; c < kMaxDof; ++c) q[c] = fmaf(s, dq[c], qa[c]);
                t = fmaf(s, dtt, ta);
            } else {
#pragma unroll
                for (int c = 0; c < kMaxDof; ++c) q[c] = 0.f;
            }
            const bool hit = state_hits<KIND, OT, OBS, FIRST>(sc, lds, q, t, act, group_mask, lower_mask);
            const uint64_t hm = __ballot(hit && act) & group_mask;
            if (!done && hm) {
                hit_at = (int32_t)(c0 + (__builtin_ctzll(hm) - gsel * lpe));
                done = true;
            }
            if (!done && c0 + lpe > n) done = true;
            if (__ballot(!done) == 0) break;
        }
        if (sub == 0 && e < E && !(valid && !valid[e])) {
            free_out[e] = hit_at < 0 ? 1 : 0;
            if (fh_out) fh_out[e] = hit_at;
            if (work) {
                // algorithmic work: the states up to the first hit, all n+1 when free
                atomicAdd(&work[0], 1ull);
                atomicAdd(&work[1], (unsigned long long)(hit_at < 0 ? n + 1 : hit_at + 1));
            }
        }
    }
}

static int ot_for(int O_pad) {
    if (O_pad <= 4) return 4;
    if (O_pad <= 8) return 8;
    if (O_pad <= 16) return 16;
    return 32;
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls f(IC<KIND>, IC<OT>, IC<OBS>) for the scene's robot kind, obstacle tile
// and obstacle-time mode.
template <class F>
static void dispatch_scene(const SceneDev &sc, F &&f) {
    auto by_ot = [&](auto kind, auto obs) {
        switch (ot_for(sc.O_pad)) {
            case 4: f(kind, IC<4>{}, obs); break;
            case 8: f(kind, IC<8>{}, obs); break;
            case 16: f(kind, IC<16>{}, obs); break;
            default: f(kind, IC<32>{}, obs); break;
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

hipError_t launch_check_edges(const SceneDev &sc, int64_t E, const float *xa, const float *xb, const uint8_t *valid,
                              uint8_t *free_out, int32_t *first_hit, int lpe_shift, hipStream_t s,
                              unsigned long long *work) {
    if (E <= 0) return hipSuccess;
    const int G = 64 >> lpe_shift;
    const int64_t per_block = 4 * (int64_t)G;
    const int64_t want = (E + per_block - 1) / per_block;
    const int blocks = (int)(want < 16384 ? want : 16384);
    const size_t lds = scene_lds_bytes(sc);
    dispatch_scene(sc, [&](auto kind, auto ot, auto obs) {
        constexpr int K = decltype(kind)::value, T = decltype(ot)::value, B = decltype(obs)::value;
        if (first_hit)
            k_check_edges<K, T, B, true><<<dim3(blocks), dim3(256), lds, s>>>(sc, E, xa, xb, valid, free_out,
                                                                             first_hit, lpe_shift, work);
        else
            k_check_edges<K, T, B, false><<<dim3(blocks), dim3(256), lds, s>>>(sc, E, xa, xb, valid, free_out,
                                                                              (int32_t *)nullptr, lpe_shift, work);
    });
    return hipGetLastError();
}

}  // namespace st
