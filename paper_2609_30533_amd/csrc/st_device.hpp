// st_device.hpp -- device-side data layout and collision primitives (gfx950).
//
// Layout in HBM (all owned by the problem handle):
//   scene:  spheres sorted by link [S] float4 (x, y, z, r); the pair table
//           R2[s][o] = (r_s + r_o + eps)^2 (-1 for padding obstacles); the obstacle
//           segment table [O_pad][n_seg][2] float4 pre-scaled by -2:
//           (-2 p_k, t_k) and (-2 v_k, span_k); waypoint times [O_pad][n_seg+1].
//   trees:  SoA x[d+1][total] (configuration rows, then time), parent[total],
//           cost[total], rootT[total]; pool p occupies [base(p), base(p)+cap(p)).
//
// The collision test keeps one space-time state per lane.  Forward kinematics
// runs in registers with the DH constants from the kernel arguments; sphere
// offsets and the pair table are staged in LDS and read as broadcasts;
// obstacle centres at the lane's own time come from the segment table, also
// staged in LDS.  A pair collides iff
//   |c|^2 + |o|^2 - 2 c.o < (r_s + r_o)^2,
// evaluated as a_s + b_o + c.n with n = -2 o (four FMA-class ops and a compare).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

constexpr int kMaxDof = 7;
constexpr int kWave = 64;

enum { kTranslate = 0, kDH = 1 };
enum { kObsShared = 0, kObsGeneric = 1 };

// Every robot/obstacle pair is tested against (r_s + r_o + kClearanceEps)^2:
// a state accepted in single precision then also clears the contact distance
// in double precision (the FP32 error of a sphere centre is ~1e-6 m).
constexpr double kClearanceEps = 2e-5;

struct SceneDev {
    int d, kind, S, O, O_pad, n_seg, obs_mode, lds_f4;  // lds_f4: float4 slots staged in LDS
    int lds_sph, lds_r2, lds_t;  // float4 offsets in LDS of the spheres, the pair table, the times
    int ot;                      // obstacles per register tile (4, 8 or 16; divides O_pad)
    float v, H, h, inv_h;
    double v_d, h_d;
    float q_lo[8], q_hi[8], q_s[8], q_g[8];
    float dh_a[8], dh_ca[8], dh_sa[8], dh_d[8], dh_t0[8];
    int link_first[9];          // spheres of link l are [link_first[l], link_first[l+1])
    const float4 *sph;          // [S]
    const float *R2;            // [S][O_pad]
    const float4 *seg;          // [O_pad][n_seg][2]
    const float *seg_t;         // shared mode: [n_seg+1]; generic: [O_pad][n_seg+1]
};

// Stage the scene into LDS: obstacle segment table, robot spheres, pair table
// and (generic mode) waypoint times.  Every thread of the block must call it.
__device__ __forceinline__ void stage_obstacles(const SceneDev &sc, float4 *lds) {
    const int n = sc.O_pad * sc.n_seg * 2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = sc.seg[i];
    for (int i = threadIdx.x; i < sc.S; i += blockDim.x) lds[sc.lds_sph + i] = sc.sph[i];
    float *r2 = reinterpret_cast<float *>(lds + sc.lds_r2);
    for (int i = threadIdx.x; i < sc.S * sc.O_pad; i += blockDim.x) r2[i] = sc.R2[i];
    if (sc.obs_mode == kObsGeneric) {
        float *lt = reinterpret_cast<float *>(lds + sc.lds_t);
        const int m = sc.O_pad * (sc.n_seg + 1);
        for (int i = threadIdx.x; i < m; i += blockDim.x) lt[i] = sc.seg_t[i];
    }
    __syncthreads();
}

// Segment index for time t with waypoint times shared by all obstacles:
// the number of interior waypoint times <= t.
__device__ __forceinline__ int shared_segment(const SceneDev &sc, float t) {
    int k = 0;
    for (int j = 1; j < sc.n_seg; ++j) k += (t >= sc.seg_t[j]) ? 1 : 0;
    return k;
}

// -2 * (obstacle centre at time t), from the pre-scaled segment table.
__device__ __forceinline__ void obstacle_n(const float4 *lds, int n_seg, int o, int k, float t, float &nx, float &ny,
                                           float &nz) {
    const float4 A = lds[(o * n_seg + k) * 2];
    const float4 B = lds[(o * n_seg + k) * 2 + 1];
    const float s = __builtin_amdgcn_fmed3f(t - A.w, 0.0f, B.w);
    nx = fmaf(s, B.x, A.x);
    ny = fmaf(s, B.y, A.y);
    nz = fmaf(s, B.z, A.z);
}

__device__ __forceinline__ int generic_segment(const SceneDev &sc, const float4 *lds, int o, float t) {
    const float *lt = reinterpret_cast<const float *>(lds + sc.lds_t) + o * (sc.n_seg + 1);
    int k = 0;
    for (int j = 1; j < sc.n_seg; ++j) k += (t >= lt[j]) ? 1 : 0;
    return k;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Sphere s (centre c, a_s = |c|^2) against the OT obstacles of the tile:
// a_s + b_o + c.n < (r_s + r_o)^2 for any o.  The radii row is read as float4
// broadcasts; each compare's lane mask (the ballot of the active lanes) is
// OR-ed on the scalar unit, so the loop is straight-line code with one add,
// three FMAs and one compare per pair.  Returns the wave mask of hits.
template <int OT>
__device__ __forceinline__ uint64_t pair_hits(const float4 *lds, const SceneDev &sc, int s, int tile, float cx,
                                              float cy, float cz, float as, const float *nx, const float *ny,
                                              const float *nz, const float *bo) {
    const float4 *r4 = reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(lds + sc.lds_r2) +
                                                        s * sc.O_pad + tile);
    float r2[OT];
#pragma unroll
    for (int i = 0; i < OT / 4; ++i) {
        const float4 v = r4[i];
        r2[4 * i] = v.x;
        r2[4 * i + 1] = v.y;
        r2[4 * i + 2] = v.z;
        r2[4 * i + 3] = v.w;
    }
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < OT; ++i) {
        float v = as + bo[i];
        v = fmaf(cx, nx[i], v);
        v = fmaf(cy, ny[i], v);
        v = fmaf(cz, nz[i], v);
        m |= __ballot(v < r2[i]);
    }
    return m;
}

// Does the lane's state (q, t) collide?  OT obstacles are held in registers
// per tile.  `alive` enters true for lanes that must check; after every link
// the wave ballots the hits and each lane decides whether it may stop:
//   FIRST:  stop on an own hit, or when a lower lane of its group has hit
//           (so the least colliding index of a group is exact);
//   !FIRST: stop as soon as any lane of its group has hit.
// Every lane of the wave must call this (it contains ballots).
template <int KIND, int OT, int OBS, bool FIRST>
__device__ __forceinline__ bool state_hits(const SceneDev &sc, const float4 *lds, const float *q, float t, bool alive,
                                           uint64_t group_mask, uint64_t lower_mask) {
    bool hit = false;
    uint64_t hm = 0;  // wave mask of lanes with a colliding pair
    // configuration box and horizon
    if (alive) {
        bool out = !(t >= 0.0f) || !(t <= sc.H);
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j)
            if (j < sc.d) out = out || !(q[j] >= sc.q_lo[j]) || !(q[j] <= sc.q_hi[j]);
        hit = out;
    }
    {
        const uint64_t m = __ballot(hit);
        if (FIRST) alive = alive && !hit && !(m & lower_mask);
        else alive = alive && !(m & group_mask);
    }
    int kseg = 0;
    if (OBS == kObsShared) kseg = shared_segment(sc, t);
    for (int tile = 0; tile < sc.O_pad; tile += OT) {
        if (__ballot(alive) == 0) break;
        float nx[OT], ny[OT], nz[OT], bo[OT];
        if (alive) {
#pragma unroll
            for (int i = 0; i < OT; ++i) {
                const int o = tile + i;
                const int k = (OBS == kObsShared) ? kseg : generic_segment(sc, lds, o, t);
                obstacle_n(lds, sc.n_seg, o, k, t, nx[i], ny[i], nz[i]);
                bo[i] = 0.25f * fmaf(nx[i], nx[i], fmaf(ny[i], ny[i], nz[i] * nz[i]));
            }
        }
        if (KIND == kTranslate) {
            const float px = q[0], py = q[1], pz = sc.d >= 3 ? q[2] : 0.0f;
            for (int s = 0; s < sc.S; ++s) {
                if (alive) {
                    const float4 sp = lds[sc.lds_sph + s];
                    const float cx = px + sp.x, cy = py + sp.y, cz = pz + sp.z;
                    const float as = fmaf(cx, cx, fmaf(cy, cy, cz * cz));
                    hm |= pair_hits<OT>(lds, sc, s, tile, cx, cy, cz, as, nx, ny, nz, bo);
                }
            }
            hit = hit || ((hm >> lane_id()) & 1ull);
            const uint64_t m = __ballot(hit);
            if (FIRST) alive = alive && !hit && !(m & lower_mask);
            else alive = alive && !(m & group_mask);
        } else {
            // world <- link frame: rotation R (row-major) and origin p
            float R00 = 1.f, R01 = 0.f, R02 = 0.f, R10 = 0.f, R11 = 1.f, R12 = 0.f, R20 = 0.f, R21 = 0.f, R22 = 1.f;
            float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
            for (int l = 0; l <= kMaxDof; ++l) {
                if (l > sc.d) break;
                if (l > 0 && alive) {
                    // T <- T * Rz(theta) Tz(d) Tx(a) Rx(alpha)
                    float st_, ct;
                    __sincosf(q[l - 1] + sc.dh_t0[l - 1], &st_, &ct);
                    const float ca = sc.dh_ca[l - 1], sa = sc.dh_sa[l - 1];
                    const float a = sc.dh_a[l - 1], dd = sc.dh_d[l - 1];
                    float u, w;
                    u = fmaf(R00, ct, R01 * st_); w = fmaf(R01, ct, -R00 * st_);
                    p0 = fmaf(a, u, fmaf(dd, R02, p0));
                    R00 = u; R01 = fmaf(ca, w, sa * R02); R02 = fmaf(ca, R02, -sa * w);
                    u = fmaf(R10, ct, R11 * st_); w = fmaf(R11, ct, -R10 * st_);
                    p1 = fmaf(a, u, fmaf(dd, R12, p1));
                    R10 = u; R11 = fmaf(ca, w, sa * R12); R12 = fmaf(ca, R12, -sa * w);
                    u = fmaf(R20, ct, R21 * st_); w = fmaf(R21, ct, -R20 * st_);
                    p2 = fmaf(a, u, fmaf(dd, R22, p2));
                    R20 = u; R21 = fmaf(ca, w, sa * R22); R22 = fmaf(ca, R22, -sa * w);
                }
                const int s0 = sc.link_first[l], s1 = sc.link_first[l + 1];
                if (s1 > s0 && __ballot(alive) != 0) {
                    for (int s = s0; s < s1; ++s) {
                        if (alive) {
                            const float4 sp = lds[sc.lds_sph + s];
                            const float cx = fmaf(R00, sp.x, fmaf(R01, sp.y, fmaf(R02, sp.z, p0)));
                            const float cy = fmaf(R10, sp.x, fmaf(R11, sp.y, fmaf(R12, sp.z, p1)));
                            const float cz = fmaf(R20, sp.x, fmaf(R21, sp.y, fmaf(R22, sp.z, p2)));
                            const float as = fmaf(cx, cx, fmaf(cy, cy, cz * cz));
                            hm |= pair_hits<OT>(lds, sc, s, tile, cx, cy, cz, as, nx, ny, nz, bo);
                        }
                    }
                    hit = hit || ((hm >> lane_id()) & 1ull);
                    const uint64_t m = __ballot(hit);
                    if (FIRST) alive = alive && !hit && !(m & lower_mask);
                    else alive = alive && !(m & group_mask);
                }
            }
        }
    }
    return hit;
}

}  // namespace st
