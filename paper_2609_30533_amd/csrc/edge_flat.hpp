// edge_flat.hpp -- edge-check building blocks shared by the collision
// translation unit and the extension pipeline: endpoint rows, the state count
// of a discretised edge, and the flattened check of short edges.
#pragma once

#include "st_internal.hpp"

namespace st {

// Both endpoint rows of edge e (rows of d + 1 floats: configuration, then
// time), earlier time first.  All the row loads are issued before the first
// use; a loop that consumed each element as it arrived would wait for every
// load in turn.
__device__ __forceinline__ void load_edge_rows(const float *xa, const float *xb, int64_t e, int d,
                                               float (&A)[kMaxDof + 1], float (&B)[kMaxDof + 1]) {
    const float *pa = xa + e * (d + 1), *pb = xb + e * (d + 1);
#pragma unroll
    for (int j = 0; j <= kMaxDof; ++j) {
        A[j] = j <= d ? pa[j] : 0.f;
        B[j] = j <= d ? pb[j] : 0.f;
    }
    if (A[d] > B[d]) {
#pragma unroll
        for (int j = 0; j <= kMaxDof; ++j) {
            const float tmp = A[j];
            A[j] = B[j];
            B[j] = tmp;
        }
    }
}

// States of a discretised edge (Eq. 5 spacing): n = ceil(max(|dq|, v dt) / h),
// at least 1; the count is taken in double precision.
__device__ __forceinline__ int32_t edge_states(const float (&A)[kMaxDof + 1], const float (&B)[kMaxDof + 1], int d,
                                               double v, double h) {
    double D2 = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxDof; ++j) {
        if (j < d) {
            const double dq = (double)B[j] - (double)A[j];
            D2 += dq * dq;
        }
    }
    const double span = fmax(sqrt(D2), v * ((double)B[d] - (double)A[d]));
    int64_t n = (int64_t)ceil(span / h);
    if (n < 1) n = 1;
    if (n > (1ll << 30)) n = 1ll << 30;
    return (int32_t)n;
}

// ---------------------------------------------------------------------------
// Short edges, flattened: a block of kFlatWaves waves takes kFlatGroups x
// a.flat consecutive edges, lays their states end to end (edge after edge,
// state order inside an edge) in rounds of 64, and decides them completely:
// state count, checks, free / first hit and the work counters, in one kernel.
// The rounds are dealt to the block's waves in turn (wave w takes rounds w,
// w + kFlatWaves, ...), so the state checks spread evenly over the CU's SIMDs
// (two waves each, so that one's memory waits overlap the other's arithmetic)
// whatever the edges' lengths; the scene is staged into LDS once per block.
// A lane skips a state above a hit already found for its edge (by any wave);
// within a round the lanes of one edge form the group of the FIRST rule, and
// hits merge with an atomic minimum, so the least colliding index is exact.
// Meant for edges of bounded length (extensions).
// ---------------------------------------------------------------------------

constexpr int kFlatEdges = 8;  // edges per wave at most (a.flat of them)
constexpr int kFlatWaves = 8;  // waves per block (two per SIMD)
constexpr int kFlatGroups = 4;  // the edges of a block: kFlatGroups x a.flat
constexpr int kFlatBlockEdges = kFlatEdges * kFlatGroups;

template <int KIND, int OT, int OBS, class Rows>
__device__ __forceinline__ void edge_flat_body(const EdgeArgs &a, float4 *lds, int bx, Rows &&rows) {
    __shared__ float s_A[kFlatBlockEdges][kMaxDof + 1], s_B[kFlatBlockEdges][kMaxDof + 1];
    __shared__ int32_t s_off[kFlatBlockEdges + 1], s_n[kFlatBlockEdges], s_hit[kFlatBlockEdges];
    const SceneDev &sc = a.sc;
    const int d = sc.d;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int NE = a.flat * kFlatGroups;  // edges of this block
    const int64_t e0 = (int64_t)bx * NE;
    // the edges' rows first (rows(e, A, B) fills both endpoints, earlier
    // time first, and returns false for an edge not to check), so that the
    // producer's loads are in flight while other threads stage the scene;
    // the staging's barrier also publishes the rows
    if (tid < kFlatBlockEdges) {
        const int64_t e = e0 + tid;
        int32_t n = -1;
        if (tid < NE && e < a.E) {
            float A[kMaxDof + 1], B[kMaxDof + 1];
            if (rows(e, A, B)) {
                n = edge_states(A, B, d, sc.v_d, sc.h_d);
#pragma unroll
                for (int j = 0; j <= kMaxDof; ++j) {
                    s_A[tid][j] = A[j];
                    s_B[tid][j] = B[j];
                }
            }
        }
        s_n[tid] = n;
        s_hit[tid] = kNoHit;
    }
    stage_obstacles(sc, lds);
    if (tid < 64) {
        // exclusive prefix of the state counts (kFlatBlockEdges <= 64 lanes)
        const int c = tid < kFlatBlockEdges ? (s_n[tid] >= 0 ? s_n[tid] + 1 : 0) : 0;
        int incl = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        if (tid < kFlatBlockEdges) s_off[tid] = incl - c;
        if (tid == kFlatBlockEdges - 1) s_off[kFlatBlockEdges] = incl;
    }
    __syncthreads();
    const int total = s_off[kFlatBlockEdges];
    for (int base = wv * 64; base < total; base += 64 * kFlatWaves) {
        const int g = base + lane;
        // edge of state g: the number of edge starts at or below g, minus one
        int i = 0;
        for (int k = 1; k < kFlatBlockEdges; ++k) i += g >= s_off[k] ? 1 : 0;
        const int j = g - s_off[i];
        const int32_t n = s_n[i];
        // a state above a known hit of its edge is not needed
        const bool act = g < total && j <= __atomic_load_n(&s_hit[i], __ATOMIC_RELAXED);
        // lanes of this edge in this round: its group for the FIRST rule
        const int lo = max(s_off[i] - base, 0), hi = min(s_off[i + 1] - base, 64);
        const uint64_t seg = (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull)) & ~((1ull << lo) - 1ull);
        const uint64_t lower = seg & ((1ull << lane) - 1ull);
        float q[kMaxDof];
        float t = 0.f;
        if (act && j == n) {
            // the last state is the endpoint itself
#pragma unroll
            for (int k = 0; k < kMaxDof; ++k) q[k] = k < d ? s_B[i][k] : 0.f;
            t = s_B[i][d];
        } else if (act) {
            const float sj = (float)j * (1.0f / (float)n);
#pragma unroll
            for (int k = 0; k < kMaxDof; ++k) q[k] = k < d ? fmaf(sj, s_B[i][k] - s_A[i][k], s_A[i][k]) : 0.f;
            t = fmaf(sj, s_B[i][d] - s_A[i][d], s_A[i][d]);
        } else {
#pragma unroll
            for (int k = 0; k < kMaxDof; ++k) q[k] = 0.f;
        }
        const bool hit = state_hits<KIND, OT, OBS, true>(sc, lds, q, t, act, seg, lower);
        if (hit && act) atomicMin(&s_hit[i], j);
    }
    __syncthreads();
    // results and work counters
    unsigned long long states = 0, edges = 0;
    if (tid < NE && tid < kFlatBlockEdges) {
        const int64_t e = e0 + tid;
        const int32_t n = s_n[tid];
        if (e < a.E && n >= 0) {
            const int32_t h = s_hit[tid];
            const bool fr = h == kNoHit;
            a.free_out[e] = fr ? 1 : 0;
            if (a.first_hit) a.first_hit[e] = fr ? -1 : h;
            states = fr ? (unsigned long long)n + 1ull : (unsigned long long)h + 1ull;
            edges = 1;
        }
    }
    if (a.work && wv == 0) {
        for (int o = 32; o > 0; o >>= 1) {
            states += __shfl_down(states, o, 64);
            edges += __shfl_down(edges, o, 64);
        }
        if (lane == 0 && edges) {
            atomicAdd(&a.work[0], edges);
            atomicAdd(&a.work[1], states);
        }
    }
}


// Blocks of the flattened path for E edges.
inline int flat_blocks(int64_t E, int edges_per_block) {
    const int64_t per = (int64_t)edges_per_block * kFlatGroups;
    return (int)((E + per - 1) / per);
}

}  // namespace st
