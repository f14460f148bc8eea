// st_device.hpp -- device-side data layout and collision primitives (gfx950).
//
// Layout in HBM (all owned by the problem handle):
//   scene:  spheres sorted by link [S] float4 (x, y, z, r); obstacle radii
//           [O_pad] (0 for padding obstacles); the obstacle segment table
//           [O_pad][n_seg][2] float4 pre-scaled by -2: (-2 p_k, t_k) and
//           (-2 v_k, span_k); waypoint times [O_pad][n_seg+1].
//   trees:  SoA x[d+1][total] (configuration rows, then time), parent[total],
//           cost[total], rootT[total]; pool p occupies [base(p), base(p)+cap(p)).
//
// The collision test keeps one space-time state per lane.  Forward kinematics
// runs in registers with the DH constants from the kernel arguments; sphere
// offsets are staged in LDS and read as broadcasts; obstacle centres at the
// lane's own time come from the segment table, also staged in LDS.  A pair
// collides iff |c - o| < r_s + r_o + eps, evaluated in expanded form as a
// minimum over the obstacle tile (sphere_clear).
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace st {

constexpr int kMaxDof = 7;
constexpr int kWave = 64;

// Robot kinds as kernel template arguments: kDHStatic is an arm whose state
// test also covers its listed link pairs and the fixed boxes.
enum { kTranslate = 0, kDH = 1, kDHStatic = 2 };
enum { kObsShared = 0, kObsGeneric = 1 };

// Every robot/obstacle pair is tested against (r_s + r_o + kClearanceEps)^2:
// a state accepted in single precision then also clears the contact distance
// in double precision (the FP32 error of a sphere centre is ~1e-6 m).
constexpr double kClearanceEps = 2e-5;

struct SceneDev {
    int d, kind, S, O, O_pad, n_seg, obs_mode, lds_f4;  // lds_f4: float4 slots staged in LDS
    int lds_sph, lds_t;         // float4 offsets in LDS of the spheres and the waypoint times
    int ot;                      // obstacles per register tile (4, 8 or 16; divides O_pad)
    float v, H, h, inv_h;
    double v_d, h_d;
    float q_lo[8], q_hi[8], q_s[8], q_g[8];
    float dh_a[8], dh_ca[8], dh_sa[8], dh_d[8], dh_t0[8];
    int link_first[9];          // spheres of link l are [link_first[l], link_first[l+1])
    int lds_goal;               // float4 offset in LDS of the sphere centres at q_g
    // static geometry (arms): self_mask[lb] bit la = link pair (la, lb) tested;
    // boxes as 4 float4 rows: (axis_a, -axis_a . centre) for a = 0..2, then
    // (half extents, 0).  goal_blocked: q_g fails the static terms.
    int stat, n_box, lds_box, goal_blocked;
    unsigned self_mask[kMaxDof + 1];
    float4 lbs[kMaxDof + 1];    // per link: bounding sphere of its spheres (link frame centre, radius)
    const float4 *box;          // [n_box][4]
    const float4 *sph;          // [S]
    const float4 *goal;         // [S] world centres at q_g (x, y, z, |c|^2)
    const float *obs_r;         // [O] obstacle radii (the continuous check)
    const float *ro;            // [O_pad] obstacle radii (0 for padding obstacles)
    float r_uni;                // the common obstacle radius, or -1 when radii differ
    const float4 *seg;          // [O_pad][n_seg][2]
    const float *seg_t;         // shared mode: [n_seg+1]; generic: [O_pad][n_seg+1]
};

// Stage the scene into LDS: obstacle segment table, robot spheres, (generic
// mode) waypoint times, the sphere centres at q_g and the fixed boxes.  Every thread of the block must call it.
__device__ __forceinline__ void stage_obstacles(const SceneDev &sc, float4 *lds) {
    const int t = threadIdx.x, bd = blockDim.x;
    const int n = sc.O_pad * sc.n_seg * 2;
    const int m = sc.obs_mode == kObsGeneric ? sc.O_pad * (sc.n_seg + 1) : 0;
    const int ng = sc.goal ? sc.S : 0, nb = 4 * sc.n_box;
    float *lt = reinterpret_cast<float *>(lds + sc.lds_t);
    // each thread's first element of every section: all the global loads are
    // in flight together before the first LDS write (section after section,
    // each write would wait for its own load in turn)
    float4 v0, v1, v2, v3;
    float v4;
    if (t < n) v0 = sc.seg[t];
    if (t < sc.S) v1 = sc.sph[t];
    if (t < ng) v2 = sc.goal[t];
    if (t < nb) v3 = sc.box[t];
    if (t < m) v4 = sc.seg_t[t];
    if (t < n) lds[t] = v0;
    if (t < sc.S) lds[sc.lds_sph + t] = v1;
    if (t < ng) lds[sc.lds_goal + t] = v2;
    if (t < nb) lds[sc.lds_box + t] = v3;
    if (t < m) lt[t] = v4;
    // sections longer than the block
    for (int i = t + bd; i < n; i += bd) lds[i] = sc.seg[i];
    for (int i = t + bd; i < sc.S; i += bd) lds[sc.lds_sph + i] = sc.sph[i];
    for (int i = t + bd; i < ng; i += bd) lds[sc.lds_goal + i] = sc.goal[i];
    for (int i = t + bd; i < nb; i += bd) lds[sc.lds_box + i] = sc.box[i];
    for (int i = t + bd; i < m; i += bd) lt[i] = sc.seg_t[i];
    __syncthreads();
}

// World frame of a link of the chain: rotation (row-major) and origin.
struct Frame {
    float R00, R01, R02, R10, R11, R12, R20, R21, R22, p0, p1, p2;
};

__device__ __forceinline__ void frame_identity(Frame &f) {
    f.R00 = 1.f; f.R01 = 0.f; f.R02 = 0.f;
    f.R10 = 0.f; f.R11 = 1.f; f.R12 = 0.f;
    f.R20 = 0.f; f.R21 = 0.f; f.R22 = 1.f;
    f.p0 = 0.f; f.p1 = 0.f; f.p2 = 0.f;
}

// T <- T * Rz(theta_j + q_j) Tz(d_j) Tx(a_j) Rx(alpha_j) (standard DH, joint j).
__device__ __forceinline__ void dh_compose(const SceneDev &sc, int j, float qj, Frame &f) {
    float st_, ct;
    __sincosf(qj + sc.dh_t0[j], &st_, &ct);
    const float ca = sc.dh_ca[j], sa = sc.dh_sa[j];
    const float a = sc.dh_a[j], dd = sc.dh_d[j];
    float u, w;
    u = fmaf(f.R00, ct, f.R01 * st_); w = fmaf(f.R01, ct, -f.R00 * st_);
    f.p0 = fmaf(a, u, fmaf(dd, f.R02, f.p0));
    f.R00 = u; f.R01 = fmaf(ca, w, sa * f.R02); f.R02 = fmaf(ca, f.R02, -sa * w);
    u = fmaf(f.R10, ct, f.R11 * st_); w = fmaf(f.R11, ct, -f.R10 * st_);
    f.p1 = fmaf(a, u, fmaf(dd, f.R12, f.p1));
    f.R10 = u; f.R11 = fmaf(ca, w, sa * f.R12); f.R12 = fmaf(ca, f.R12, -sa * w);
    u = fmaf(f.R20, ct, f.R21 * st_); w = fmaf(f.R21, ct, -f.R20 * st_);
    f.p2 = fmaf(a, u, fmaf(dd, f.R22, f.p2));
    f.R20 = u; f.R21 = fmaf(ca, w, sa * f.R22); f.R22 = fmaf(ca, f.R22, -sa * w);
}

// Frame of link b expressed in the frame of link a: R = Ra^T Rb,
// p = Ra^T (pb - pa).
__device__ __forceinline__ void frame_relative(const Frame &a, const Frame &b, Frame &m) {
    m.R00 = fmaf(a.R00, b.R00, fmaf(a.R10, b.R10, a.R20 * b.R20));
    m.R01 = fmaf(a.R00, b.R01, fmaf(a.R10, b.R11, a.R20 * b.R21));
    m.R02 = fmaf(a.R00, b.R02, fmaf(a.R10, b.R12, a.R20 * b.R22));
    m.R10 = fmaf(a.R01, b.R00, fmaf(a.R11, b.R10, a.R21 * b.R20));
    m.R11 = fmaf(a.R01, b.R01, fmaf(a.R11, b.R11, a.R21 * b.R21));
    m.R12 = fmaf(a.R01, b.R02, fmaf(a.R11, b.R12, a.R21 * b.R22));
    m.R20 = fmaf(a.R02, b.R00, fmaf(a.R12, b.R10, a.R22 * b.R20));
    m.R21 = fmaf(a.R02, b.R01, fmaf(a.R12, b.R11, a.R22 * b.R21));
    m.R22 = fmaf(a.R02, b.R02, fmaf(a.R12, b.R12, a.R22 * b.R22));
    const float dx = b.p0 - a.p0, dy = b.p1 - a.p1, dz = b.p2 - a.p2;
    m.p0 = fmaf(a.R00, dx, fmaf(a.R10, dy, a.R20 * dz));
    m.p1 = fmaf(a.R01, dx, fmaf(a.R11, dy, a.R21 * dz));
    m.p2 = fmaf(a.R02, dx, fmaf(a.R12, dy, a.R22 * dz));
}

// World centre of a sphere given in its link frame, and |c|^2.
__device__ __forceinline__ void sphere_world(const Frame &f, float4 sp, float &cx, float &cy, float &cz, float &as) {
    cx = fmaf(f.R00, sp.x, fmaf(f.R01, sp.y, fmaf(f.R02, sp.z, f.p0)));
    cy = fmaf(f.R10, sp.x, fmaf(f.R11, sp.y, fmaf(f.R12, sp.z, f.p1)));
    cz = fmaf(f.R20, sp.x, fmaf(f.R21, sp.y, fmaf(f.R22, sp.z, f.p2)));
    as = fmaf(cx, cx, fmaf(cy, cy, cz * cz));
}

// Translating robot: centre = (q0, q1, q2 or 0) + offset, and |c|^2.
__device__ __forceinline__ void sphere_translate(const SceneDev &sc, const float *q, float4 sp, float &cx, float &cy,
                                                 float &cz, float &as) {
    const float pz = sc.d >= 3 ? q[2] : 0.0f;
    cx = q[0] + sp.x;
    cy = q[1] + sp.y;
    cz = pz + sp.z;
    as = fmaf(cx, cx, fmaf(cy, cy, cz * cz));
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

// Sphere (centre c, a_s = |c|^2, radius r_s) against the OT obstacles of the
// tile.  With n = -2 o and A_o = |o|^2 - r_o^2 (per lane and obstacle, at the
// lane's time), a pair collides iff
//   A_o + c.n - 2 r r_o < r^2 - a_s,   r = r_s + eps,
// which is |c - o|^2 < (r + r_o)^2 expanded.  The loop keeps the minimum of
// the left side over the tile (three or four FMAs and half a min3 per pair,
// no scalar-unit work); the result is that minimum minus the right side,
// negative iff some pair collides.  With equal obstacle radii (UNI) the
// r_o term moves to the right side.
template <int OT, bool UNI>
__device__ __forceinline__ float sphere_clear(const SceneDev &sc, float cx, float cy, float cz, float as, float r_s,
                                              const float *nx, const float *ny, const float *nz, const float *A,
                                              const float *ro) {
    const float r = r_s + (float)kClearanceEps;
    const float k = -2.0f * r;
    float m = INFINITY;
#pragma unroll
    for (int i = 0; i < OT; ++i) {
        float v = fmaf(cx, nx[i], A[i]);
        v = fmaf(cy, ny[i], v);
        v = fmaf(cz, nz[i], v);
        if (!UNI) v = fmaf(k, ro[i], v);
        m = fminf(m, v);
    }
    float rhs = fmaf(r, r, -as);
    if (UNI) rhs = fmaf(-k, sc.r_uni, rhs);
    return m - rhs;
}

// Squared distance from point c to fixed box b: offsets along the box axes,
// their excess over the half extents (zero inside), and the squared norm.
__device__ __forceinline__ float box_dist2(const float4 *lds, const SceneDev &sc, int b, float cx, float cy,
                                           float cz) {
    const float4 *B = lds + sc.lds_box + 4 * b;
    const float4 a0 = B[0], a1 = B[1], a2 = B[2], hb = B[3];
    const float u0 = fmaf(a0.x, cx, fmaf(a0.y, cy, fmaf(a0.z, cz, a0.w)));
    const float u1 = fmaf(a1.x, cx, fmaf(a1.y, cy, fmaf(a1.z, cz, a1.w)));
    const float u2 = fmaf(a2.x, cx, fmaf(a2.y, cy, fmaf(a2.z, cz, a2.w)));
    const float e0 = fmaxf(fabsf(u0) - hb.x, 0.0f);
    const float e1 = fmaxf(fabsf(u1) - hb.y, 0.0f);
    const float e2 = fmaxf(fabsf(u2) - hb.z, 0.0f);
    return fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
}

// Spheres [s0, s1) of link b, offsets p_b, against spheres [a0, a1) of link a,
// with m the frame of b in the frame of a: a pair collides iff
// |m p_b - p_a| < r_a + r_b + eps.  `first` is this lane's first sphere of b
// and `step` its stride (the lane split of a state).
__device__ __forceinline__ bool link_pair_hits(const float4 *lds, const SceneDev &sc, const Frame &m, int first,
                                               int s1, int step, int a0, int a1) {
    bool h = false;
    for (int s = first; s < s1; s += step) {
        const float4 sp = lds[sc.lds_sph + s];
        const float cx = fmaf(m.R00, sp.x, fmaf(m.R01, sp.y, fmaf(m.R02, sp.z, m.p0)));
        const float cy = fmaf(m.R10, sp.x, fmaf(m.R11, sp.y, fmaf(m.R12, sp.z, m.p1)));
        const float cz = fmaf(m.R20, sp.x, fmaf(m.R21, sp.y, fmaf(m.R22, sp.z, m.p2)));
        const float rb = sp.w + (float)kClearanceEps;
        for (int a = a0; a < a1; ++a) {
            const float4 pa = lds[sc.lds_sph + a];
            const float dx = cx - pa.x, dy = cy - pa.y, dz = cz - pa.z;
            const float R = pa.w + rb;
            h = h || fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < R * R;
        }
    }
    return h;
}

// Broad phase of the static terms: a link's spheres lie inside its bounding
// sphere (centre and radius per link, in the link frame); when two bounding
// spheres, or a bounding sphere and a box, are more than kBroadMargin apart,
// every sphere pair between them clears contact by that much and the exact
// tests are skipped (they could only report free).
constexpr float kBroadMargin = 1e-3f;

template <int SPLIT>
__device__ __forceinline__ bool state_hit(uint64_t hm, int st_lane);

// Self-collision of the listed link pairs and the fixed boxes for the lane's
// configuration q (time-independent).  Every link frame is kept in
// registers; per link, the spheres near a box are tested against it in the
// world frame and, per listed lower link whose bound is near, against that
// link's spheres in its frame (one relative transform per link pair).
// Updates hit / hm / alive as the obstacle tiles do.  Every lane of the wave
// must call this.
template <bool FIRST, int SPLIT>
__device__ __forceinline__ void static_pass(const SceneDev &sc, const float4 *lds, const float *q, bool &alive,
                                            bool &hit, uint64_t &hm, uint64_t group_mask, uint64_t lower_mask,
                                            int part, int st_lane) {
    Frame F[kMaxDof + 1];
    frame_identity(F[0]);
#pragma unroll
    for (int l = 0; l <= kMaxDof; ++l) {
        if (l > sc.d) break;
        if (l > 0) {
            F[l] = F[l - 1];
            if (alive) dh_compose(sc, l - 1, q[l - 1], F[l]);
        }
        if (__ballot(alive) == 0) break;
        const int s0 = sc.link_first[l], s1 = sc.link_first[l + 1];
        if (s1 <= s0) continue;
        const int first = s0 + ((part - s0) & (SPLIT - 1));
        const float4 bl = sc.lbs[l];
        bool h = false;
        if (sc.n_box > 0 && alive) {
            float bx, by, bz, bs;
            sphere_world(F[l], bl, bx, by, bz, bs);
            const float rb = bl.w + kBroadMargin;
            for (int b = 0; b < sc.n_box; ++b) {
                if (box_dist2(lds, sc, b, bx, by, bz) < rb * rb) {
                    for (int s = first; s < s1; s += SPLIT) {
                        float cx, cy, cz, as;
                        const float4 sp = lds[sc.lds_sph + s];
                        sphere_world(F[l], sp, cx, cy, cz, as);
                        const float rr = sp.w + (float)kClearanceEps;
                        h = h || box_dist2(lds, sc, b, cx, cy, cz) < rr * rr;
                    }
                }
            }
        }
#pragma unroll
        for (int la = 0; la < kMaxDof; ++la) {
            if (la >= l) break;
            const int a0 = sc.link_first[la], a1 = sc.link_first[la + 1];
            if (!((sc.self_mask[l] >> la) & 1u) || a1 <= a0) continue;
            if (alive) {
                Frame m;
                frame_relative(F[la], F[l], m);
                const float4 ba = sc.lbs[la];
                const float dx = fmaf(m.R00, bl.x, fmaf(m.R01, bl.y, fmaf(m.R02, bl.z, m.p0))) - ba.x;
                const float dy = fmaf(m.R10, bl.x, fmaf(m.R11, bl.y, fmaf(m.R12, bl.z, m.p1))) - ba.y;
                const float dz = fmaf(m.R20, bl.x, fmaf(m.R21, bl.y, fmaf(m.R22, bl.z, m.p2))) - ba.z;
                const float R = ba.w + bl.w + kBroadMargin;
                if (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < R * R)
                    h = h || link_pair_hits(lds, sc, m, first, s1, SPLIT, a0, a1);
            }
        }
        hm |= __ballot(h);
        hit = hit || state_hit<SPLIT>(hm, st_lane);
        const uint64_t mk = __ballot(hit);
        if (FIRST) alive = alive && !hit && !(mk & lower_mask);
        else alive = alive && !(mk & group_mask);
    }
}

// Hit of the lane's state from the lane's accumulated pair masks.  A lane
// knows its own bit exactly (its own ballots included it); with SPLIT > 1
// the lanes of a state ran different numbers of sphere iterations, so their
// own bits are exchanged by one more ballot of the whole wave.  Every lane of
// the wave must call this.
template <int SPLIT>
__device__ __forceinline__ bool state_hit(uint64_t hm, int st_lane) {
    if (SPLIT == 1) return (hm >> lane_id()) & 1ull;
    const uint64_t own = __ballot(((hm >> lane_id()) & 1ull) != 0);
    return ((own >> st_lane) & ((1ull << SPLIT) - 1ull)) != 0;
}

// Does the lane's state (q, t) collide?  OT obstacles are held in registers
// per tile.  With SPLIT > 1 a state occupies SPLIT adjacent lanes (aligned)
// and lane `part` of them tests the spheres s with s = part (mod SPLIT);
// every lane composes the kinematic chain itself, and a state's hit is the OR
// over its lanes, so all SPLIT lanes return the same answer.  This divides
// the dependent chain of one state check by about SPLIT for launches too
// small to fill the device.  `alive` enters true for lanes that must check;
// after every link the wave ballots the hits and each lane decides whether it
// may stop:
//   FIRST:  stop on a hit of its state, or when a lower state of its group
//           has hit (so the least colliding index of a group is exact);
//           lower_mask holds the lanes of the lower states;
//   !FIRST: stop as soon as any lane of its group has hit.
// Every lane of the wave must call this (it contains ballots).
template <int KIND, int OT, int OBS, bool FIRST, int SPLIT = 1>
__device__ __forceinline__ bool state_hits(const SceneDev &sc, const float4 *lds, const float *q, float t, bool alive,
                                           uint64_t group_mask, uint64_t lower_mask, int part = 0) {
    static_assert(SPLIT == 1 || SPLIT == 2 || SPLIT == 4 || SPLIT == 8, "state split");
    const int st_lane = lane_id() & ~(SPLIT - 1);  // first lane of this state
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
        float nx[OT], ny[OT], nz[OT], A[OT], ro[OT];
#pragma unroll
        for (int i = 0; i < OT; ++i) ro[i] = sc.ro[tile + i];
        if (alive) {
#pragma unroll
            for (int i = 0; i < OT; ++i) {
                const int o = tile + i;
                const int k = (OBS == kObsShared) ? kseg : generic_segment(sc, lds, o, t);
                obstacle_n(lds, sc.n_seg, o, k, t, nx[i], ny[i], nz[i]);
                A[i] = fmaf(0.25f, fmaf(nx[i], nx[i], fmaf(ny[i], ny[i], nz[i] * nz[i])), -ro[i] * ro[i]);
            }
        }
        // one specialisation for equal obstacle radii, one for mixed radii
        auto run = [&](auto uni_c) {
            constexpr bool UNI = decltype(uni_c)::value;
            if (KIND == kTranslate) {
                float dmin = INFINITY;
                for (int s = part; s < sc.S; s += SPLIT) {
                    if (alive) {
                        float cx, cy, cz, as;
                        const float4 sp = lds[sc.lds_sph + s];
                        sphere_translate(sc, q, sp, cx, cy, cz, as);
                        dmin = fminf(dmin, sphere_clear<OT, UNI>(sc, cx, cy, cz, as, sp.w, nx, ny, nz, A, ro));
                    }
                }
                hm |= __ballot(alive && dmin < 0.0f);
                hit = hit || state_hit<SPLIT>(hm, st_lane);
                const uint64_t m = __ballot(hit);
                if (FIRST) alive = alive && !hit && !(m & lower_mask);
                else alive = alive && !(m & group_mask);
            } else {
                // world <- link frame
                Frame f;
                frame_identity(f);
#pragma unroll
                for (int l = 0; l <= kMaxDof; ++l) {
                    if (l > sc.d) break;
                    if (l > 0 && alive) dh_compose(sc, l - 1, q[l - 1], f);
                    const int s0 = sc.link_first[l], s1 = sc.link_first[l + 1];
                    if (s1 > s0 && __ballot(alive) != 0) {
                        // broad phase for links of three spheres or more: the
                        // link's bounding sphere (its spheres' radii included)
                        // clearing every obstacle of the tile by kBroadMargin
                        // clears each of its spheres (the margin is far above
                        // the FP32 error), so the pair tests decide the same;
                        // the wave skips the link when all its lanes clear it
                        bool need = alive;
                        if (alive && s1 - s0 >= 3) {
                            const float4 bl = sc.lbs[l];
                            float bx, by, bz, bs;
                            sphere_world(f, make_float4(bl.x, bl.y, bl.z, 0.0f), bx, by, bz, bs);
                            need = sphere_clear<OT, UNI>(sc, bx, by, bz, bs, bl.w + kBroadMargin, nx, ny, nz, A, ro) <
                                   0.0f;
                        }
                        // this lane's spheres of the link: s = part (mod SPLIT)
                        float dmin = INFINITY;
                        if (__ballot(need) != 0 && need) {
                            // two spheres per step: both offset reads are in flight together
                            const int first = s0 + ((part - s0) & (SPLIT - 1));
                            int s = first;
                            for (; s + SPLIT < s1; s += 2 * SPLIT) {
                                const float4 sp = lds[sc.lds_sph + s];
                                const float4 sq = lds[sc.lds_sph + s + SPLIT];
                                float cx, cy, cz, as, ex, ey, ez, bs;
                                sphere_world(f, sp, cx, cy, cz, as);
                                sphere_world(f, sq, ex, ey, ez, bs);
                                dmin = fminf(dmin, sphere_clear<OT, UNI>(sc, cx, cy, cz, as, sp.w, nx, ny, nz, A, ro));
                                dmin = fminf(dmin, sphere_clear<OT, UNI>(sc, ex, ey, ez, bs, sq.w, nx, ny, nz, A, ro));
                            }
                            if (s < s1) {
                                const float4 sp = lds[sc.lds_sph + s];
                                float cx, cy, cz, as;
                                sphere_world(f, sp, cx, cy, cz, as);
                                dmin = fminf(dmin, sphere_clear<OT, UNI>(sc, cx, cy, cz, as, sp.w, nx, ny, nz, A, ro));
                            }
                        }
                        hm |= __ballot(alive && dmin < 0.0f);
                        hit = hit || state_hit<SPLIT>(hm, st_lane);
                        const uint64_t m = __ballot(hit);
                        if (FIRST) alive = alive && !hit && !(m & lower_mask);
                        else alive = alive && !(m & group_mask);
                    }
                }
            }
        };
        if (sc.r_uni >= 0.0f) run(std::true_type{});
        else run(std::false_type{});
    }
    // time-independent terms for the lanes still undecided
    if (KIND == kDHStatic && __ballot(alive) != 0)
        static_pass<FIRST, SPLIT>(sc, lds, q, alive, hit, hm, group_mask, lower_mask, part, st_lane);
    return hit;
}

// Does (q_g, t) collide?  The same decision as state_hits at q = q_g, with
// the sphere centres at q_g read from LDS (they are computed once per
// problem by the same kinematics code), so only the obstacle positions at t
// and the pair tests remain; the static terms at q_g are decided once per
// problem by the state test itself (goal_blocked).  SPLIT lanes share a state as in state_hits;
// lanes are independent otherwise (`alive` false: nothing to check).
template <int OT, int OBS, int SPLIT>
__device__ __forceinline__ bool goal_hits(const SceneDev &sc, const float4 *lds, float t, bool alive, int part) {
    const int st_lane = lane_id() & ~(SPLIT - 1);
    bool hit = false;
    uint64_t hm = 0;
    if (alive) {
        bool out = !(t >= 0.0f) || !(t <= sc.H) || sc.goal_blocked;
#pragma unroll
        for (int j = 0; j < kMaxDof; ++j)
            if (j < sc.d) out = out || !(sc.q_g[j] >= sc.q_lo[j]) || !(sc.q_g[j] <= sc.q_hi[j]);
        hit = out;
    }
    alive = alive && !hit;
    int kseg = 0;
    if (OBS == kObsShared) kseg = shared_segment(sc, t);
    for (int tile = 0; tile < sc.O_pad; tile += OT) {
        if (__ballot(alive) == 0) break;
        float nx[OT], ny[OT], nz[OT], A[OT], ro[OT];
#pragma unroll
        for (int i = 0; i < OT; ++i) ro[i] = sc.ro[tile + i];
        if (alive) {
#pragma unroll
            for (int i = 0; i < OT; ++i) {
                const int o = tile + i;
                const int k = (OBS == kObsShared) ? kseg : generic_segment(sc, lds, o, t);
                obstacle_n(lds, sc.n_seg, o, k, t, nx[i], ny[i], nz[i]);
                A[i] = fmaf(0.25f, fmaf(nx[i], nx[i], fmaf(ny[i], ny[i], nz[i] * nz[i])), -ro[i] * ro[i]);
            }
        }
        for (int l = 0; l <= sc.d; ++l) {
            const int s0 = sc.link_first[l], s1 = sc.link_first[l + 1];
            if (s1 > s0 && __ballot(alive) != 0) {
                float dmin = INFINITY;
                for (int s = s0 + ((part - s0) & (SPLIT - 1)); s < s1; s += SPLIT) {
                    if (alive) {
                        const float4 c = lds[sc.lds_goal + s];
                        const float r_s = lds[sc.lds_sph + s].w;
                        dmin = fminf(dmin, sphere_clear<OT, false>(sc, c.x, c.y, c.z, c.w, r_s, nx, ny, nz, A, ro));
                    }
                }
                hm |= __ballot(alive && dmin < 0.0f);
                hit = hit || state_hit<SPLIT>(hm, st_lane);
                alive = alive && !hit;
            }
        }
    }
    return hit;
}

}  // namespace st
