// api.hip -- C ABI entry points: problem lifecycle, scene upload, goal grid,
// collision queries and state I/O.  The planner pipeline lives in extend.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <numeric>

#include "pipeline.hpp"
#include "st_internal.hpp"

namespace st {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static bool finite(double x) { return std::isfinite(x); }

static int ot_of(int O) {
    if (O <= 4) return 4;
    if (O <= 8) return 8;
    return 16;
}

template <class T>
static int dev_upload(T **dst, const T *src, size_t n) {
    if (n == 0) n = 1;
    ST_HIP(hipMalloc((void **)dst, n * sizeof(T)));
    if (src) ST_HIP(hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice));
    return ST_OK;
}

static int validate(const st_problem_desc *D) {
    if (!D) return fail(ST_EINVAL, "null description");
    const int d = D->dof;
    if (d < 1 || d > ST_MAX_DOF) return fail(ST_EINVAL, "dof %d outside 1..%d", d, ST_MAX_DOF);
    if (D->robot_kind != ST_ROBOT_TRANSLATE && D->robot_kind != ST_ROBOT_DH)
        return fail(ST_EINVAL, "unknown robot kind %d", D->robot_kind);
    if (D->robot_kind == ST_ROBOT_TRANSLATE && (d < 2 || d > 3))
        return fail(ST_EINVAL, "a translating robot needs dof 2 or 3");
    if (D->robot_kind == ST_ROBOT_DH && !D->dh) return fail(ST_EINVAL, "DH robot without a DH table");
    if (D->n_spheres < 1 || D->n_spheres > ST_MAX_SPHERES) return fail(ST_EINVAL, "n_spheres %d", D->n_spheres);
    if (!D->sphere_link || !D->spheres) return fail(ST_EINVAL, "missing sphere arrays");
    if (!D->q_lo || !D->q_hi || !D->q_start || !D->q_goal) return fail(ST_EINVAL, "missing configuration arrays");
    for (int s = 0; s < D->n_spheres; ++s) {
        const int l = D->sphere_link[s];
        if (l < 0 || l > (D->robot_kind == ST_ROBOT_DH ? d : 0)) return fail(ST_EINVAL, "sphere %d link %d", s, l);
        for (int c = 0; c < 4; ++c)
            if (!finite(D->spheres[4 * s + c])) return fail(ST_EINVAL, "sphere %d not finite", s);
        if (D->spheres[4 * s + 3] < 0) return fail(ST_EINVAL, "negative sphere radius");
    }
    if (D->robot_kind == ST_ROBOT_DH)
        for (int i = 0; i < 4 * d; ++i)
            if (!finite(D->dh[i])) return fail(ST_EINVAL, "DH table not finite");
    for (int j = 0; j < d; ++j) {
        const double lo = D->q_lo[j], hi = D->q_hi[j];
        if (!finite(lo) || !finite(hi) || !(lo < hi)) return fail(ST_EINVAL, "bad box in dimension %d", j);
        if (!finite(D->q_start[j]) || !finite(D->q_goal[j])) return fail(ST_EINVAL, "start/goal not finite");
        if (D->q_start[j] < lo || D->q_start[j] > hi) return fail(ST_EINVAL, "start outside C (dimension %d)", j);
        if (D->q_goal[j] < lo || D->q_goal[j] > hi) return fail(ST_EINVAL, "goal outside C (dimension %d)", j);
    }
    if (!finite(D->t_min) || !finite(D->t_max) || D->t_min > D->t_max || D->t_max <= 0)
        return fail(ST_EINVAL, "bad arrival range [%g, %g]", D->t_min, D->t_max);
    if (!finite(D->v_max) || !(D->v_max > 0)) return fail(ST_EINVAL, "v_max must be > 0");
    if (D->n_obstacles < 0 || D->n_obstacles > ST_MAX_OBSTACLES) return fail(ST_EINVAL, "n_obstacles %d", D->n_obstacles);
    if (D->n_obstacles > 0) {
        if (!D->n_waypoints || !D->waypoints || !D->obstacle_radius) return fail(ST_EINVAL, "missing obstacle arrays");
        if (D->max_waypoints < 1 || D->max_waypoints > ST_MAX_WAYPOINTS)
            return fail(ST_EINVAL, "max_waypoints %d", D->max_waypoints);
        for (int o = 0; o < D->n_obstacles; ++o) {
            const int n = D->n_waypoints[o];
            if (n < 1 || n > D->max_waypoints) return fail(ST_EINVAL, "obstacle %d has %d waypoints", o, n);
            if (!finite(D->obstacle_radius[o]) || D->obstacle_radius[o] < 0)
                return fail(ST_EINVAL, "obstacle %d radius", o);
            const double *w = D->waypoints + (size_t)o * D->max_waypoints * 4;
            for (int k = 0; k < n; ++k) {
                for (int c = 0; c < 4; ++c)
                    if (!finite(w[4 * k + c])) return fail(ST_EINVAL, "obstacle %d waypoint %d not finite", o, k);
                if (k > 0 && w[4 * k] < w[4 * (k - 1)]) return fail(ST_EINVAL, "obstacle %d times decrease", o);
            }
        }
    }
    if (D->n_self_pairs < 0 || D->n_self_pairs > ST_MAX_SELF_PAIRS)
        return fail(ST_EINVAL, "n_self_pairs %d outside 0..%d", D->n_self_pairs, ST_MAX_SELF_PAIRS);
    if (D->n_boxes < 0 || D->n_boxes > ST_MAX_BOXES) return fail(ST_EINVAL, "n_boxes %d outside 0..%d", D->n_boxes, ST_MAX_BOXES);
    if ((D->n_self_pairs > 0 || D->n_boxes > 0) && D->robot_kind != ST_ROBOT_DH)
        return fail(ST_EINVAL, "self pairs and boxes are defined for arms (ST_ROBOT_DH)");
    if (D->n_self_pairs > 0 && !D->self_pairs) return fail(ST_EINVAL, "missing self pair array");
    for (int k = 0; k < D->n_self_pairs; ++k) {
        const int la = D->self_pairs[2 * k], lb = D->self_pairs[2 * k + 1];
        if (la < 0 || la >= lb || lb > d) return fail(ST_EINVAL, "self pair %d = (%d, %d) needs 0 <= la < lb <= %d", k, la, lb, d);
    }
    if (D->n_boxes > 0 && !D->boxes) return fail(ST_EINVAL, "missing box array");
    for (int b = 0; b < D->n_boxes; ++b) {
        const double *B = D->boxes + 15 * b;
        for (int c = 0; c < 15; ++c)
            if (!finite(B[c])) return fail(ST_EINVAL, "box %d not finite", b);
        for (int c = 3; c < 6; ++c)
            if (B[c] < 0) return fail(ST_EINVAL, "box %d has a negative half extent", b);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double *u = B + 6 + 3 * i, *v = B + 6 + 3 * j;
                const double dot = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
                if (fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-6) return fail(ST_EINVAL, "box %d axes not orthonormal", b);
            }
    }
    const st_params &P = D->params;
    if (P.variant != ST_INTERVAL_ROOT && P.variant != ST_ROOT_RECYCLING) return fail(ST_EINVAL, "variant %d", P.variant);
    if (P.no_recycling != 0 && P.no_recycling != 1) return fail(ST_EINVAL, "no_recycling %d", P.no_recycling);
    if (P.obstacle_tile != 0 && P.obstacle_tile != 4 && P.obstacle_tile != 8 && P.obstacle_tile != 16)
        return fail(ST_EINVAL, "obstacle_tile %d (0, 4, 8 or 16)", P.obstacle_tile);
    if (P.n_groups < 1 || P.n_groups > ST_MAX_GROUPS) return fail(ST_EINVAL, "n_groups %d", P.n_groups);
    if (P.batch < 1) return fail(ST_EINVAL, "batch %d", P.batch);
    if (!(P.eta > 0) || !(P.h > 0) || !(P.dt > 0) || !finite(P.eta) || !finite(P.h) || !finite(P.dt))
        return fail(ST_EINVAL, "eta, h and dt must be positive");
    if (!(P.p_new >= 0 && P.p_new <= 1) || !(P.p_guided >= 0 && P.p_guided <= 1))
        return fail(ST_EINVAL, "probabilities outside [0, 1]");
    if (P.cap_fwd < 2 || P.cap_bwd < 2) return fail(ST_EINVAL, "capacities must be >= 2");
    const double total = (double)P.cap_fwd + (double)P.n_groups * P.cap_bwd;
    if (total > 2147483647.0) return fail(ST_EINVAL, "total capacity exceeds 2^31 - 1 nodes");
    if (D->t_max / P.dt > 1e8) return fail(ST_EINVAL, "goal grid too fine");
    return ST_OK;
}

// Obstacle segment table, pre-scaled by -2 (see st_device.hpp).
static int build_scene(st_problem *p, const st_problem_desc *D) {
    const int d = D->dof, S = D->n_spheres, O = D->n_obstacles;
    SceneDev &sc = p->sc;
    memset(&sc, 0, sizeof sc);
    sc.d = d;
    sc.kind = D->robot_kind == ST_ROBOT_DH ? kDH : kTranslate;
    sc.S = S;
    sc.O = O;
    const int OT = D->params.obstacle_tile > 0 ? D->params.obstacle_tile : ot_of(O);
    sc.O_pad = std::max(OT, (O + OT - 1) / OT * OT);
    sc.ot = OT;
    sc.v = (float)D->v_max;
    sc.H = (float)D->t_max;
    sc.h = (float)D->params.h;
    sc.inv_h = (float)(1.0 / D->params.h);
    sc.v_d = (double)(float)D->v_max;
    sc.h_d = D->params.h;
    for (int j = 0; j < 8; ++j) {
        sc.q_lo[j] = j < d ? (float)D->q_lo[j] : 0.f;
        sc.q_hi[j] = j < d ? (float)D->q_hi[j] : 0.f;
        sc.q_s[j] = j < d ? (float)D->q_start[j] : 0.f;
        sc.q_g[j] = j < d ? (float)D->q_goal[j] : 0.f;
        sc.dh_ca[j] = 1.f;
    }
    if (sc.kind == kDH)
        for (int j = 0; j < d; ++j) {
            const double *r = D->dh + 4 * j;
            sc.dh_a[j] = (float)r[0];
            sc.dh_ca[j] = (float)cos(r[1]);
            sc.dh_sa[j] = (float)sin(r[1]);
            sc.dh_d[j] = (float)r[2];
            sc.dh_t0[j] = (float)r[3];
        }
    // spheres sorted by link (stable)
    std::vector<int> ord(S);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return D->sphere_link[a] < D->sphere_link[b]; });
    std::vector<float4> sph(S);
    for (int i = 0; i < S; ++i) {
        const double *s = D->spheres + 4 * ord[i];
        sph[i] = make_float4((float)s[0], (float)s[1], (float)s[2], (float)s[3]);
    }
    // obstacle radii padded with zeros; the common radius when all agree
    std::vector<float> ro((size_t)sc.O_pad, 0.0f);
    sc.r_uni = O > 0 ? (float)D->obstacle_radius[0] : -1.0f;
    for (int o = 0; o < O; ++o) {
        ro[o] = (float)D->obstacle_radius[o];
        if (ro[o] != sc.r_uni) sc.r_uni = -1.0f;
    }
    for (int l = 0; l <= 8; ++l) {
        int c = 0;
        for (int i = 0; i < S; ++i)
            if (D->sphere_link[ord[i]] < l) ++c;
        sc.link_first[l] = c;
    }
    // do all obstacles share their waypoint times?
    bool shared = O > 0;
    for (int o = 1; o < O && shared; ++o) {
        if (D->n_waypoints[o] != D->n_waypoints[0]) shared = false;
        for (int k = 0; k < D->n_waypoints[0] && shared; ++k)
            if (D->waypoints[((size_t)o * D->max_waypoints + k) * 4] != D->waypoints[(size_t)k * 4]) shared = false;
    }
    if (O == 0) shared = true;
    int nseg = 1;
    for (int o = 0; o < O; ++o) nseg = std::max(nseg, D->n_waypoints[o] - 1);
    sc.n_seg = nseg;
    sc.obs_mode = shared ? kObsShared : kObsGeneric;
    std::vector<float4> seg((size_t)sc.O_pad * nseg * 2);
    std::vector<float> segt;
    if (shared) segt.assign(nseg + 1, 0.f);
    else segt.assign((size_t)sc.O_pad * (nseg + 1), 0.f);
    for (int o = 0; o < sc.O_pad; ++o) {
        const double *w = o < O ? D->waypoints + (size_t)o * D->max_waypoints * 4 : nullptr;
        const int n = o < O ? D->n_waypoints[o] : 1;
        for (int k = 0; k < nseg; ++k) {
            double px, py, pz, tk, vx = 0, vy = 0, vz = 0, span = 0;
            if (!w) {
                px = py = pz = 1e3;
                tk = 0;
            } else if (k + 1 < n) {
                const double *a = w + 4 * k, *b = w + 4 * (k + 1);
                tk = a[0];
                px = a[1];
                py = a[2];
                pz = a[3];
                span = b[0] - a[0];
                if (span > 0) {
                    vx = (b[1] - a[1]) / span;
                    vy = (b[2] - a[2]) / span;
                    vz = (b[3] - a[3]) / span;
                }
            } else {
                const double *a = w + 4 * (n - 1);
                tk = a[0];
                px = a[1];
                py = a[2];
                pz = a[3];
            }
            seg[((size_t)o * nseg + k) * 2] = make_float4((float)(-2 * px), (float)(-2 * py), (float)(-2 * pz), (float)tk);
            seg[((size_t)o * nseg + k) * 2 + 1] =
                make_float4((float)(-2 * vx), (float)(-2 * vy), (float)(-2 * vz), (float)span);
        }
        // waypoint times (interior times drive the segment search)
        for (int k = 0; k <= nseg; ++k) {
            float tv;
            if (!w) tv = 0.f;
            else if (k < n) tv = (float)w[4 * k];
            else tv = INFINITY;
            if (shared) {
                if (o == 0) segt[k] = tv;
            } else {
                segt[(size_t)o * (nseg + 1) + k] = tv;
            }
        }
    }
    if (shared && O == 0) segt.assign(nseg + 1, INFINITY);
    // LDS: segment table, spheres, waypoint times (generic mode), goal centres, boxes
    sc.lds_sph = sc.O_pad * nseg * 2;
    sc.lds_t = sc.lds_sph + S;
    sc.lds_goal = sc.lds_t + (shared ? 0 : (int)((segt.size() + 3) / 4));
    sc.lds_box = sc.lds_goal + S;
    sc.lds_f4 = sc.lds_box + 4 * D->n_boxes;
    // static geometry: link-pair masks and boxes as (axis, -axis . centre) rows
    sc.n_box = D->n_boxes;
    for (int k = 0; k < D->n_self_pairs; ++k) sc.self_mask[D->self_pairs[2 * k + 1]] |= 1u << D->self_pairs[2 * k];
    sc.stat = (D->n_self_pairs > 0 || D->n_boxes > 0) ? 1 : 0;
    // per-link bounding spheres of the broad phase: centroid of the link's
    // sphere centres, radius the farthest sphere surface, rounded outwards
    for (int l = 0; l <= d && l <= kMaxDof; ++l) {
        double c[3] = {0, 0, 0};
        int n = 0;
        for (int i = 0; i < S; ++i)
            if (D->sphere_link[ord[i]] == l) {
                for (int k = 0; k < 3; ++k) c[k] += D->spheres[4 * ord[i] + k];
                ++n;
            }
        if (n == 0) continue;
        for (int k = 0; k < 3; ++k) c[k] /= n;
        const float cf[3] = {(float)c[0], (float)c[1], (float)c[2]};
        double rho = 0;
        for (int i = 0; i < S; ++i)
            if (D->sphere_link[ord[i]] == l) {
                const double *sp = D->spheres + 4 * ord[i];
                const double e = sqrt((sp[0] - cf[0]) * (sp[0] - cf[0]) + (sp[1] - cf[1]) * (sp[1] - cf[1]) +
                                      (sp[2] - cf[2]) * (sp[2] - cf[2]));
                rho = std::max(rho, e + sp[3]);
            }
        sc.lbs[l] = make_float4(cf[0], cf[1], cf[2], (float)(rho * (1.0 + 1e-6) + 1e-6));
    }
    int rc;
    if ((rc = dev_upload(&p->d_sph, sph.data(), sph.size())) != ST_OK) return rc;
    if ((rc = dev_upload(&p->d_ro, ro.data(), ro.size())) != ST_OK) return rc;
    if ((rc = dev_upload(&p->d_seg, seg.data(), seg.size())) != ST_OK) return rc;
    if ((rc = dev_upload(&p->d_segt, segt.data(), segt.size())) != ST_OK) return rc;
    sc.sph = p->d_sph;
    sc.ro = p->d_ro;
    sc.seg = p->d_seg;
    sc.seg_t = p->d_segt;
    // obstacle radii for the continuous check
    {
        std::vector<float> radii((size_t)std::max(O, 1), 0.f);
        for (int o = 0; o < O; ++o) radii[o] = (float)D->obstacle_radius[o];
        if ((rc = dev_upload(&p->d_obs_r, radii.data(), radii.size())) != ST_OK) return rc;
        sc.obs_r = p->d_obs_r;
    }
    if (D->n_boxes > 0) {
        std::vector<float4> bx((size_t)4 * D->n_boxes);
        for (int b = 0; b < D->n_boxes; ++b) {
            const double *B = D->boxes + 15 * b;
            for (int a = 0; a < 3; ++a) {
                const double *u = B + 6 + 3 * a;
                const double w = -(u[0] * B[0] + u[1] * B[1] + u[2] * B[2]);
                bx[4 * b + a] = make_float4((float)u[0], (float)u[1], (float)u[2], (float)w);
            }
            bx[4 * b + 3] = make_float4((float)B[3], (float)B[4], (float)B[5], 0.f);
        }
        if ((rc = dev_upload(&p->d_box, bx.data(), bx.size())) != ST_OK) return rc;
        sc.box = p->d_box;
    }
    // sphere centres at q_g for the goal-state tests
    ST_HIP(hipMalloc((void **)&p->d_goal, std::max(S, 1) * sizeof(float4)));
    sc.goal = nullptr;
    ST_HIP(launch_goal_centers(sc, p->d_goal));
    ST_HIP(hipDeviceSynchronize());
    sc.goal = p->d_goal;
    if (scene_lds_bytes(sc) > 64 * 1024) return fail(ST_EINVAL, "obstacle table too large for LDS");
    // the static terms at q_g, decided once by the state test itself with the
    // moving obstacles left out
    sc.goal_blocked = 0;
    if (sc.stat) {
        SceneDev s2 = sc;
        s2.O = 0;
        s2.O_pad = 0;
        float xg[kMaxDof + 1];
        for (int j = 0; j < d; ++j) xg[j] = sc.q_g[j];
        xg[d] = 0.f;
        float *dx = nullptr;
        uint8_t *dfree = nullptr, hfree = 0;
        ST_HIP(hipMalloc((void **)&dx, sizeof xg));
        ST_HIP(hipMalloc((void **)&dfree, 1));
        ST_HIP(hipMemcpy(dx, xg, (d + 1) * sizeof(float), hipMemcpyHostToDevice));
        ST_HIP(launch_check_states(s2, 1, dx, dfree, 0));
        ST_HIP(hipMemcpy(&hfree, dfree, 1, hipMemcpyDeviceToHost));
        ST_HIP(hipFree(dx));
        ST_HIP(hipFree(dfree));
        sc.goal_blocked = hfree ? 0 : 1;
    }
    return ST_OK;
}

// Goal grid valid(q_g, k dt) for k in [ceil(L/dt), floor(H/dt)] (Eq. 5) and
// the merged guided windows [k_a dt - dt/2, k_b dt + dt/2] clipped to [L, H].
static int build_goal_grid(st_problem *p) {
    const double dt = p->prm.dt;
    p->k_lo = (int64_t)ceil(p->L / dt);
    p->k_hi = (int64_t)floor(p->t_max / dt);
    const int64_t nk = std::max<int64_t>(p->k_hi - p->k_lo + 1, 0);
    p->h_gfree.assign((size_t)std::max<int64_t>(nk, 1), 0);
    if ((size_t)nk > 0) {
        std::vector<float> xs((size_t)nk * (p->d + 1));
        for (int64_t k = 0; k < nk; ++k) {
            for (int j = 0; j < p->d; ++j) xs[(size_t)k * (p->d + 1) + j] = (float)p->q_g[j];
            xs[(size_t)k * (p->d + 1) + p->d] = (float)((double)(p->k_lo + k) * dt);
        }
        float *dx = nullptr;
        ST_HIP(hipMalloc((void **)&dx, xs.size() * sizeof(float)));
        ST_HIP(hipMalloc((void **)&p->d_gfree, (size_t)nk));
        ST_HIP(hipMemcpy(dx, xs.data(), xs.size() * sizeof(float), hipMemcpyHostToDevice));
        ST_HIP(launch_check_states(p->sc, nk, dx, p->d_gfree, 0));
        ST_HIP(hipMemcpy(p->h_gfree.data(), p->d_gfree, (size_t)nk, hipMemcpyDeviceToHost));
        ST_HIP(hipFree(dx));
    } else {
        ST_HIP(hipMalloc((void **)&p->d_gfree, 1));
        ST_HIP(hipMemset(p->d_gfree, 0, 1));
    }
    p->h_wlo.clear();
    p->h_whi.clear();
    for (int64_t k = p->k_lo; k <= p->k_hi; ++k) {
        if (!p->h_gfree[(size_t)(k - p->k_lo)]) continue;
        int64_t k2 = k;
        while (k2 + 1 <= p->k_hi && p->h_gfree[(size_t)(k2 + 1 - p->k_lo)]) ++k2;
        const double lo = std::max(k * dt - dt / 2.0, p->L);
        const double hi = std::min(k2 * dt + dt / 2.0, p->t_max);
        if (hi > lo) {
            p->h_wlo.push_back(lo);
            p->h_whi.push_back(hi);
        }
        k = k2;
    }
    p->h_wcum.assign(p->h_wlo.size() + 1, 0.0);
    for (size_t j = 0; j < p->h_wlo.size(); ++j) p->h_wcum[j + 1] = p->h_wcum[j] + (p->h_whi[j] - p->h_wlo[j]);
    int rc;
    if ((rc = dev_upload(&p->d_wlo, p->h_wlo.data(), p->h_wlo.size())) != ST_OK) return rc;
    if ((rc = dev_upload(&p->d_whi, p->h_whi.data(), p->h_whi.size())) != ST_OK) return rc;
    if ((rc = dev_upload(&p->d_wcum, p->h_wcum.data(), p->h_wcum.size())) != ST_OK) return rc;
    WindowsDev &w = p->win;
    w.lo = p->d_wlo;
    w.hi = p->d_whi;
    w.cum = p->d_wcum;
    w.nw = (int32_t)p->h_wlo.size();
    w.L = p->L;
    w.H = p->t_max;
    w.dt = dt;
    w.N = p->prm.n_groups;
    w.k_lo = (int32_t)p->k_lo;
    w.k_hi = (int32_t)p->k_hi;
    w.gfree = p->d_gfree;
    return ST_OK;
}

static int alloc_trees(st_problem *p) {
    TreeDev &t = p->tree;
    t.d = p->d;
    t.cap_fwd = p->prm.cap_fwd;
    t.cap_bwd = p->prm.cap_bwd;
    t.n_pools = 1 + p->prm.n_groups;
    t.total = (int64_t)t.cap_fwd + (int64_t)p->prm.n_groups * t.cap_bwd;
    ST_HIP(hipMalloc((void **)&t.x, (size_t)t.total * (p->d + 1) * sizeof(float)));
    ST_HIP(hipMalloc((void **)&t.parent, (size_t)t.total * sizeof(int32_t)));
    ST_HIP(hipMalloc((void **)&t.cost, (size_t)t.total * sizeof(float)));
    ST_HIP(hipMalloc((void **)&t.rootT, (size_t)t.total * sizeof(float)));
    ST_HIP(hipMalloc((void **)&p->d_plan, sizeof(PlanDev)));
    return ST_OK;
}

// Host helper: write one node (used at initialisation only).
static int put_node(st_problem *p, int64_t idx, const double *q, double t, int32_t parent, float cost, float rootT) {
    const TreeDev &T = p->tree;
    for (int j = 0; j <= p->d; ++j) {
        const float v = (float)(j < p->d ? q[j] : t);
        ST_HIP(hipMemcpy(T.x + (size_t)j * T.total + idx, &v, sizeof(float), hipMemcpyHostToDevice));
    }
    ST_HIP(hipMemcpy(T.parent + idx, &parent, sizeof(int32_t), hipMemcpyHostToDevice));
    ST_HIP(hipMemcpy(T.cost + idx, &cost, sizeof(float), hipMemcpyHostToDevice));
    ST_HIP(hipMemcpy(T.rootT + idx, &rootT, sizeof(float), hipMemcpyHostToDevice));
    return ST_OK;
}

// Interval root with incumbent U: Ubar = min(H, U), the guided length G below
// Ubar and the number of windows starting below it.
static void ir_alloc_host(const st_problem *p, double U, PlanDev &pl) {
    pl.Ubar = std::min(p->t_max, U);
    int j = 0;
    while (j < (int)p->h_wlo.size() && p->h_wlo[j] < pl.Ubar) ++j;
    pl.jstar = j;
    pl.G = j > 0 ? p->h_wcum[j - 1] + (std::min(p->h_whi[j - 1], pl.Ubar) - p->h_wlo[j - 1]) : 0.0;
    pl.done = !(p->L < pl.Ubar);
}

// Initial recycling roots: split the grid indices with k dt < H into N equal
// integer strata; slot j takes the first free grid time of stratum j.
static void rr_init_host(const st_problem *p, PlanDev &pl, std::vector<int64_t> &root_k) {
    const int N = p->prm.n_groups;
    int64_t k_end = p->k_hi + 1;
    while (k_end > p->k_lo && (double)(k_end - 1) * p->prm.dt >= p->t_max) --k_end;
    const int64_t K = k_end - p->k_lo;
    root_k.assign(N, -1);
    for (int s = 0; s < N; ++s) {
        pl.slot_active[s] = 0;
        pl.slotT[s] = INFINITY;
        pl.slotK[s] = -1;
        pl.slot_gen[s] = 0;
        if (K <= 0) continue;
        const int64_t a = p->k_lo + (K * s) / N, b = p->k_lo + (K * (s + 1)) / N;
        for (int64_t k = a; k < b; ++k) {
            if (!p->h_gfree[(size_t)(k - p->k_lo)]) continue;
            root_k[s] = k;
            pl.slotT[s] = (float)((double)k * p->prm.dt);
            pl.slotK[s] = (int32_t)k;
            pl.slot_active[s] = 1;
            break;
        }
    }
    pl.n_active = 0;
    for (int s = 0; s < N; ++s)
        if (pl.slot_active[s]) pl.active_list[pl.n_active++] = s;
}

static int init_state(st_problem *p) {
    PlanDev pl;
    memset(&pl, 0, sizeof pl);
    pl.U = INFINITY;
    pl.C = INFINITY;
    pl.inc_f = pl.inc_b = -1;
    pl.first_iter = -1;
    for (int g = 0; g < kMaxGroups; ++g) {
        pl.minRootT[g] = INFINITY;
        pl.slotT[g] = INFINITY;
        pl.slotK[g] = -1;
    }
    // forward root (q_s, 0)
    int rc = put_node(p, 0, p->q_s.data(), 0.0, -1, 0.f, 0.f);
    if (rc != ST_OK) return rc;
    pl.count[0] = 1;
    if (p->prm.variant == ST_INTERVAL_ROOT) {
        ir_alloc_host(p, INFINITY, pl);
    } else {
        std::vector<int64_t> rk;
        rr_init_host(p, pl, rk);
        for (int s = 0; s < p->prm.n_groups; ++s) {
            if (rk[s] < 0) continue;
            const double T = (double)rk[s] * p->prm.dt;
            rc = put_node(p, pool_base(p->tree, 1 + s), p->q_g.data(), T, -1, 0.f, (float)T);
            if (rc != ST_OK) return rc;
            pl.count[1 + s] = 1;
        }
    }
    ST_HIP(hipMemcpy(p->d_plan, &pl, sizeof pl, hipMemcpyHostToDevice));
    p->iter = 0;
    return ST_OK;
}

static void destroy(st_problem *p) {
    if (!p) return;
    graphs_free(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    work_free(p);
    edge_bufs_free(p->ebufs);
    edge_bufs_free(p->ebufs_api);
    for (hipEvent_t ev : p->prof_ev) (void)hipEventDestroy(ev);
    void *bufs[] = {p->d_sph, p->d_ro, p->d_seg, p->d_segt, p->d_goal, p->d_obs_r, p->d_box, p->d_gfree, p->d_wlo, p->d_whi, p->d_wcum,
                    p->tree.x, p->tree.parent, p->tree.cost, p->tree.rootT, p->d_plan};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

}  // namespace st

using namespace st;

extern "C" {

const char *st_last_error(void) { return g_err.c_str(); }

int st_problem_create(const st_problem_desc *D, st_problem **out) {
    if (!out) return fail(ST_EINVAL, "null output handle");
    *out = nullptr;
    int rc = validate(D);
    if (rc != ST_OK) return rc;
    st_problem *p = new (std::nothrow) st_problem();
    if (!p) return fail(ST_ENOMEM, "out of host memory");
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(ST_EHIP, "no HIP device");
    }
    p->prm = D->params;
    p->d = D->dof;
    p->kind = D->robot_kind;
    p->S = D->n_spheres;
    p->O = D->n_obstacles;
    p->q_lo.assign(D->q_lo, D->q_lo + p->d);
    p->q_hi.assign(D->q_hi, D->q_hi + p->d);
    p->q_s.assign(D->q_start, D->q_start + p->d);
    p->q_g.assign(D->q_goal, D->q_goal + p->d);
    p->t_min = D->t_min;
    p->t_max = D->t_max;
    p->v_max = D->v_max;
    double D2 = 0;
    for (int j = 0; j < p->d; ++j) D2 += (p->q_g[j] - p->q_s[j]) * (p->q_g[j] - p->q_s[j]);
    p->Lg = sqrt(D2) / p->v_max;
    p->L = std::max(p->Lg, p->t_min);
    // default lanes per edge chunk: enough for a typical steered edge
    {
        const double n_typ = p->prm.eta / p->prm.h + 1.0;
        int shift = 3;
        while ((1 << shift) < n_typ && shift < 6) ++shift;
        p->tune_ext = shift;
        p->tune_api = shift;
        // bridges mostly collide within their first few states: short chunks
        // let one wave take several bridges
        p->tune_br = 4;
    }
    if ((rc = build_scene(p, D)) != ST_OK || (rc = build_goal_grid(p)) != ST_OK || (rc = alloc_trees(p)) != ST_OK ||
        (rc = init_state(p)) != ST_OK || (rc = work_reserve(p, p->prm.batch)) != ST_OK) {
        destroy(p);
        return rc;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        destroy(p);
        return fail(ST_EHIP, "device synchronisation failed after create");
    }
    *out = p;
    g_err.clear();
    return ST_OK;
}

void st_problem_destroy(st_problem *p) { destroy(p); }

int st_problem_reset(st_problem *p) {
    if (!p) return fail(ST_EINVAL, "null problem");
    ST_HIP(hipDeviceSynchronize());
    return init_state(p);
}

int st_set_tuning(st_problem *p, int32_t obstacle_tile, int32_t lanes_extension, int32_t lanes_bridge,
                  int32_t lanes_check) {
    if (!p) return fail(ST_EINVAL, "null problem");
    auto shift_of = [](int32_t lanes, int32_t *out) {
        for (int s = 0; s <= 6; ++s)
            if ((1 << s) == lanes) {
                *out = s;
                return true;
            }
        return lanes == 0;
    };
    int32_t se = p->tune_ext, sb = p->tune_br, sk = p->tune_api;
    if (!shift_of(lanes_extension, &se) || !shift_of(lanes_bridge, &sb) || !shift_of(lanes_check, &sk))
        return fail(ST_EINVAL, "lanes must be 0 (keep) or a power of two up to 64");
    if (obstacle_tile != 0) {
        if ((obstacle_tile != 4 && obstacle_tile != 8 && obstacle_tile != 16) || p->sc.O_pad % obstacle_tile)
            return fail(ST_EINVAL, "obstacle tile must be 4, 8 or 16 and divide %d", p->sc.O_pad);
        p->sc.ot = obstacle_tile;
    }
    p->tune_ext = se;
    p->tune_br = sb;
    p->tune_api = sk;
    ST_HIP(hipDeviceSynchronize());
    graphs_free(p);
    return ST_OK;
}

int st_set_state_split(st_problem *p, int32_t split_extension, int32_t split_bridge, int32_t split_check) {
    if (!p) return fail(ST_EINVAL, "null problem");
    auto shift_of = [](int32_t v, int *out) {
        switch (v) {
            case 0: return true;
            case -1: *out = -1; return true;
            case 1: *out = 0; return true;
            case 2: *out = 1; return true;
            case 4: *out = 2; return true;
            default: return false;
        }
    };
    int se = p->split_ext, sb = p->split_br, sk = p->split_api;
    if (!shift_of(split_extension, &se) || !shift_of(split_bridge, &sb) || !shift_of(split_check, &sk))
        return fail(ST_EINVAL, "state split must be 1, 2 or 4, -1 (by launch size) or 0 (keep)");
    p->split_ext = se;
    p->split_br = sb;
    p->split_api = sk;
    ST_HIP(hipDeviceSynchronize());
    graphs_free(p);
    return ST_OK;
}

int st_set_flat_extension(st_problem *p, int32_t edges_per_block) {
    if (!p) return fail(ST_EINVAL, "null problem");
    if (edges_per_block < 0 || edges_per_block > 8)
        return fail(ST_EINVAL, "edges per block must be 0 (chunked path) to 8");
    p->flat_ext = edges_per_block;
    ST_HIP(hipDeviceSynchronize());
    graphs_free(p);
    return ST_OK;
}

int st_check_states(st_problem *p, int64_t M, const float *x, uint8_t *free_out, void *stream) {
    if (!p || M < 0 || (M > 0 && (!x || !free_out))) return fail(ST_EINVAL, "st_check_states: bad arguments");
    ST_HIP(launch_check_states(p->sc, M, x, free_out, (hipStream_t)stream));
    return ST_OK;
}

int st_check_edges(st_problem *p, int64_t E, const float *xa, const float *xb, uint8_t *free_out,
                   int32_t *first_hit, void *stream) {
    if (!p || E < 0 || (E > 0 && (!xa || !xb || !free_out))) return fail(ST_EINVAL, "st_check_edges: bad arguments");
    if (E == 0) return ST_OK;
    // separate from the planner's buffers, which captured graphs refer to
    int rc = edge_bufs_reserve(p->ebufs_api, E);
    if (rc != ST_OK) return rc;
    ST_HIP(launch_check_edges(p->sc, p->ebufs_api, E, xa, xb, nullptr, free_out, first_hit, p->tune_api,
                              (hipStream_t)stream, nullptr, split_for(p->split_api, E)));
    return ST_OK;
}

}  // extern "C"

namespace st {

// One query of a goal sequence (Sec. III): leg i starts at the previous goal
// with local time 0 at the previous arrival T, the obstacle trajectories
// shifted by T and the remaining horizon; only the last goal keeps the
// arrival range's lower end.  The description points into this object's own
// waypoint copy.
struct SequenceLeg {
    std::vector<double> wp;
    st_problem_desc D;
    // false when no horizon is left
    bool make(const st_problem_desc *desc, int32_t m, const double *goals, int i, const double *q_start,
              double T) {
        const int d = desc->dof, O = desc->n_obstacles, Wm = desc->max_waypoints;
        wp.assign(O > 0 ? (size_t)O * Wm * 4 : 1, 0.0);
        D = *desc;
        for (int o = 0; o < O; ++o)
            for (int k = 0; k < Wm; ++k) {
                const size_t r = ((size_t)o * Wm + k) * 4;
                wp[r] = desc->waypoints[r] - T;
                for (int c = 1; c < 4; ++c) wp[r + c] = desc->waypoints[r + c];
            }
        if (O > 0) D.waypoints = wp.data();
        D.q_start = q_start;
        D.q_goal = goals + (size_t)i * d;
        D.t_max = desc->t_max - T;
        D.t_min = i + 1 == m ? std::max(0.0, desc->t_min - T) : 0.0;
        D.params.problem_id = desc->params.problem_id + 7919u * (uint32_t)i;
        return D.t_max > 0.0;
    }
};

// Appends a leg's path (local time) to an absolute-time path; a leg starts
// where the previous one ended, so its first state is dropped after leg 0.
static void append_leg(std::vector<double> &states, const st_path &leg, int d, int i, double T) {
    for (int64_t s = (i > 0 ? 1 : 0); s < leg.n_states; ++s) {
        for (int j = 0; j < d; ++j) states.push_back(leg.states[s * (d + 1) + j]);
        states.push_back(leg.states[s * (d + 1) + d] + T);
    }
}

static int finish_sequence(st_path *out, const std::vector<double> &states, int d, double T, double C) {
    out->n_states = (int64_t)(states.size() / (d + 1));
    out->states = (double *)malloc(sizeof(double) * std::max<size_t>(states.size(), 1));
    if (!out->states) return fail(ST_ENOMEM, "goal sequence: out of host memory");
    memcpy(out->states, states.data(), sizeof(double) * states.size());
    out->arrival = T;
    out->length = C;
    return ST_OK;
}

}  // namespace st

extern "C" {

int st_plan_sequence(const st_problem_desc *desc, int32_t m, const double *goals, const st_budget *budget,
                     st_path *out) {
    if (!desc || m < 1 || !goals || !budget || !out) return fail(ST_EINVAL, "st_plan_sequence: bad arguments");
    memset(out, 0, sizeof *out);
    const int d = desc->dof;
    out->dof = d;
    out->first_solution_iter = -1;
    out->arrival = INFINITY;
    out->length = INFINITY;
    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    std::vector<double> qs(desc->q_start, desc->q_start + d);
    std::vector<double> states;  // absolute-time path, rows of d + 1
    double T = 0.0, C = 0.0;
    int64_t iters = 0;
    double first_ms = 0.0;
    int rc = ST_OK;
    SequenceLeg L;
    for (int i = 0; i < m && rc == ST_OK; ++i) {
        if (!L.make(desc, m, goals, i, qs.data(), T)) {
            rc = ST_NO_SOLUTION;
            break;
        }
        st_problem *p = nullptr;
        if ((rc = st_problem_create(&L.D, &p)) != ST_OK) break;
        st_path leg;
        const int lr = st_plan(p, budget, &leg);
        st_problem_destroy(p);
        if (lr < 0) {
            st_path_free(&leg);
            rc = lr;
            break;
        }
        if (lr == ST_NO_SOLUTION || leg.n_states < 1) {
            st_path_free(&leg);
            rc = ST_NO_SOLUTION;
            break;
        }
        append_leg(states, leg, d, i, T);
        T += leg.arrival;
        C += leg.length;
        iters += leg.iterations;
        first_ms += leg.first_solution_ms;
        if (i + 1 == m) {
            out->first_solution_iter = leg.first_solution_iter;
            out->first_solution_ms = first_ms;
        }
        st_path_free(&leg);
        qs.assign(goals + (size_t)i * d, goals + (size_t)(i + 1) * d);
    }
    out->iterations = iters;
    out->total_ms = ms_since();
    if (rc != ST_OK) return rc;
    return finish_sequence(out, states, d, T, C);
}

int st_plan_sequence_batch(const st_problem_desc *descs, int32_t P, const int32_t *m, const double *const *goals,
                           const st_budget *budget, st_path *outs, int32_t *rcs) {
    if (!descs || P < 1 || P > 4096 || !m || !goals || !budget || !outs || !rcs)
        return fail(ST_EINVAL, "st_plan_sequence_batch: bad arguments");
    for (int k = 0; k < P; ++k)
        if (m[k] < 1 || !goals[k]) return fail(ST_EINVAL, "st_plan_sequence_batch: problem %d has no goals", k);
    const auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    std::vector<std::vector<double>> qs(P), states(P);
    std::vector<double> T(P, 0.0), C(P, 0.0);
    int32_t max_m = 0;
    for (int k = 0; k < P; ++k) {
        memset(&outs[k], 0, sizeof outs[k]);
        outs[k].dof = descs[k].dof;
        outs[k].first_solution_iter = -1;
        outs[k].arrival = INFINITY;
        outs[k].length = INFINITY;
        qs[k].assign(descs[k].q_start, descs[k].q_start + descs[k].dof);
        rcs[k] = ST_OK;
        max_m = std::max(max_m, m[k]);
    }
    int rc = ST_OK;
    for (int i = 0; i < max_m && rc == ST_OK; ++i) {
        // leg i of every problem still on its way, planned as one batch
        std::vector<int> who;
        std::vector<SequenceLeg> legs(P);
        std::vector<st_problem *> hs;
        for (int k = 0; k < P && rc == ST_OK; ++k) {
            if (i >= m[k] || rcs[k] != ST_OK) continue;
            if (!legs[k].make(&descs[k], m[k], goals[k], i, qs[k].data(), T[k])) {
                rcs[k] = ST_NO_SOLUTION;
                continue;
            }
            st_problem *h = nullptr;
            const int r = st_problem_create(&legs[k].D, &h);
            if (r != ST_OK) {
                rc = r;
                break;
            }
            who.push_back(k);
            hs.push_back(h);
        }
        if (rc == ST_OK && !hs.empty()) {
            st_batch *b = nullptr;
            rc = st_batch_create(hs.data(), (int32_t)hs.size(), 4, &b);
            if (rc == ST_OK) {
                st_batch_result br;
                memset(&br, 0, sizeof br);
                rc = st_batch_plan(b, budget, &br);
                st_batch_destroy(b);
            }
            for (size_t j = 0; j < who.size() && rc == ST_OK; ++j) {
                const int k = who[j];
                st_path leg;
                const int lr = st_path_get(hs[j], &leg);
                if (lr < 0 && lr != ST_ECAPACITY) {
                    st_path_free(&leg);
                    rc = lr;
                    break;
                }
                if (lr != ST_OK || leg.n_states < 1) {
                    // a trivial leg (start = goal, arrival 0 allowed) has one state
                    st_problem *h = hs[j];
                    bool start_free = false, trivial = false;
                    if (lr == ST_NO_SOLUTION && start_check(h, &start_free, &trivial) == ST_OK && trivial) {
                        for (int c = 0; c < descs[k].dof; ++c) states[k].push_back(qs[k][c]);
                        states[k].push_back(T[k]);
                        if (i + 1 < m[k]) qs[k].assign(goals[k] + (size_t)i * descs[k].dof,
                                                       goals[k] + (size_t)(i + 1) * descs[k].dof);
                        st_path_free(&leg);
                        continue;
                    }
                    rcs[k] = lr == ST_ECAPACITY ? ST_ECAPACITY : ST_NO_SOLUTION;
                    st_path_free(&leg);
                    continue;
                }
                const int d = descs[k].dof;
                append_leg(states[k], leg, d, i, T[k]);
                T[k] += leg.arrival;
                C[k] += leg.length;
                outs[k].iterations += leg.iterations;
                st_path_free(&leg);
                qs[k].assign(goals[k] + (size_t)i * d, goals[k] + (size_t)(i + 1) * d);
            }
        }
        for (st_problem *h : hs) st_problem_destroy(h);
    }
    for (int k = 0; k < P; ++k) {
        outs[k].total_ms = ms_since();
        if (rc == ST_OK && rcs[k] == ST_OK) {
            const int r = finish_sequence(&outs[k], states[k], descs[k].dof, T[k], C[k]);
            if (r != ST_OK) rc = r;
        }
    }
    return rc;
}

int st_check_edges_continuous(st_problem *p, int64_t E, const float *xa, const float *xb, uint8_t *free_out,
                              float *dmin_out, void *stream) {
    if (!p || E < 0 || (E > 0 && (!xa || !xb || !free_out)))
        return fail(ST_EINVAL, "st_check_edges_continuous: bad arguments");
    if (p->kind != ST_ROBOT_TRANSLATE)
        return fail(ST_EINVAL, "st_check_edges_continuous: translating robots only");
    ST_HIP(launch_check_edges_continuous(p->sc, E, xa, xb, free_out, dmin_out, (hipStream_t)stream));
    return ST_OK;
}

int st_get_info(st_problem *p, st_info *out) {
    if (!p || !out) return fail(ST_EINVAL, "st_get_info: bad arguments");
    PlanDev pl;
    ST_HIP(hipDeviceSynchronize());
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    out->U = pl.U;
    out->C = pl.C;
    out->inc_fwd = pl.inc_f;
    out->inc_bwd = pl.inc_b;
    out->L = p->L;
    out->H = p->t_max;
    out->k_lo = p->k_lo;
    out->k_hi = p->k_hi;
    out->iter = p->iter;
    out->overflow = pl.overflow;
    out->n_active = pl.n_active;
    out->total_cap = p->tree.total;
    out->n_pools = p->tree.n_pools;
    out->first_iter = pl.first_iter;
    out->batch = p->prm.batch;
    out->obstacle_tile = p->sc.ot;
    out->lanes_extension = 1 << p->tune_ext;
    out->lanes_bridge = 1 << p->tune_br;
    out->lanes_check = 1 << p->tune_api;
    return ST_OK;
}

int st_tree_export(st_problem *p, int64_t *counts, float *x, int32_t *parent, float *cost, float *rootT) {
    if (!p) return fail(ST_EINVAL, "null problem");
    ST_HIP(hipDeviceSynchronize());
    PlanDev pl;
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    const TreeDev &T = p->tree;
    if (counts)
        for (int i = 0; i < T.n_pools; ++i) counts[i] = pl.count[i];
    if (x) {
        std::vector<float> soa((size_t)T.total * (p->d + 1));
        ST_HIP(hipMemcpy(soa.data(), T.x, soa.size() * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < T.total; ++i)
            for (int j = 0; j <= p->d; ++j) x[(size_t)i * (p->d + 1) + j] = soa[(size_t)j * T.total + i];
    }
    if (parent) ST_HIP(hipMemcpy(parent, T.parent, (size_t)T.total * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cost) ST_HIP(hipMemcpy(cost, T.cost, (size_t)T.total * sizeof(float), hipMemcpyDeviceToHost));
    if (rootT) ST_HIP(hipMemcpy(rootT, T.rootT, (size_t)T.total * sizeof(float), hipMemcpyDeviceToHost));
    return ST_OK;
}

int st_tree_import(st_problem *p, const int64_t *counts, const float *x, const int32_t *parent, const float *cost,
                   const float *rootT, double U, double C, int64_t inc_fwd, int64_t inc_bwd, int64_t iter,
                   const double *slot_T, const int32_t *slot_active, const uint32_t *slot_gen, const int64_t *slot_k) {
    if (!p || !counts || !x || !parent || !cost || !rootT) return fail(ST_EINVAL, "st_tree_import: bad arguments");
    const TreeDev &T = p->tree;
    for (int i = 0; i < T.n_pools; ++i)
        if (counts[i] < 0 || counts[i] > pool_cap(T, i)) return fail(ST_EINVAL, "pool %d count %lld", i, (long long)counts[i]);
    if (p->prm.variant == ST_ROOT_RECYCLING && (!slot_T || !slot_active || !slot_gen || !slot_k))
        return fail(ST_EINVAL, "root recycling needs the slot arrays");
    ST_HIP(hipDeviceSynchronize());
    std::vector<float> soa((size_t)T.total * (p->d + 1));
    for (int64_t i = 0; i < T.total; ++i)
        for (int j = 0; j <= p->d; ++j) soa[(size_t)j * T.total + i] = x[(size_t)i * (p->d + 1) + j];
    ST_HIP(hipMemcpy(T.x, soa.data(), soa.size() * sizeof(float), hipMemcpyHostToDevice));
    ST_HIP(hipMemcpy(T.parent, parent, (size_t)T.total * sizeof(int32_t), hipMemcpyHostToDevice));
    ST_HIP(hipMemcpy(T.cost, cost, (size_t)T.total * sizeof(float), hipMemcpyHostToDevice));
    ST_HIP(hipMemcpy(T.rootT, rootT, (size_t)T.total * sizeof(float), hipMemcpyHostToDevice));
    PlanDev pl;
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    for (int i = 0; i < T.n_pools; ++i) pl.count[i] = (int32_t)counts[i];
    pl.U = (float)U;
    pl.C = (float)C;
    pl.inc_f = (int32_t)inc_fwd;
    pl.inc_b = (int32_t)inc_bwd;
    pl.iter = (int32_t)iter;
    p->iter = iter;
    if (p->prm.variant == ST_INTERVAL_ROOT) {
        ir_alloc_host(p, U, pl);
        for (int g = 0; g < p->prm.n_groups; ++g) {
            float m = INFINITY;
            const int64_t b = pool_base(T, 1 + g);
            for (int64_t i = 0; i < counts[1 + g]; ++i)
                if (parent[b + i] < 0) m = std::min(m, rootT[b + i]);
            pl.minRootT[g] = m;
        }
    } else {
        pl.n_active = 0;
        for (int s = 0; s < p->prm.n_groups; ++s) {
            pl.slotT[s] = (float)slot_T[s];
            pl.slot_active[s] = slot_active[s];
            pl.slot_gen[s] = slot_gen[s];
            pl.slotK[s] = (int32_t)slot_k[s];
            if (slot_active[s]) pl.active_list[pl.n_active++] = s;
        }
    }
    ST_HIP(hipMemcpy(p->d_plan, &pl, sizeof pl, hipMemcpyHostToDevice));
    return ST_OK;
}

int st_slots_export(st_problem *p, double *slot_T, int32_t *slot_active, uint32_t *slot_gen, int64_t *slot_k) {
    if (!p) return fail(ST_EINVAL, "null problem");
    ST_HIP(hipDeviceSynchronize());
    PlanDev pl;
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    for (int s = 0; s < p->prm.n_groups; ++s) {
        if (slot_T) slot_T[s] = pl.slotT[s];
        if (slot_active) slot_active[s] = pl.slot_active[s];
        if (slot_gen) slot_gen[s] = pl.slot_gen[s];
        if (slot_k) slot_k[s] = pl.slotK[s];
    }
    return ST_OK;
}

int st_goal_grid_export(st_problem *p, uint8_t *free_out) {
    if (!p || !free_out) return fail(ST_EINVAL, "st_goal_grid_export: bad arguments");
    const int64_t nk = p->k_hi - p->k_lo + 1;
    if (nk > 0) memcpy(free_out, p->h_gfree.data(), (size_t)nk);
    return ST_OK;
}

int st_partition_export(st_problem *p, double *I, int32_t *n_pieces, double *pieces, int32_t maxp) {
    if (!p || !I || !n_pieces || !pieces || maxp < 1) return fail(ST_EINVAL, "st_partition_export: bad arguments");
    ST_HIP(hipDeviceSynchronize());
    PlanDev pl;
    ST_HIP(hipMemcpy(&pl, p->d_plan, sizeof pl, hipMemcpyDeviceToHost));
    const int N = p->prm.n_groups;
    const double w = (pl.Ubar - p->L) / N;
    for (int i = 0; i < N; ++i) {
        I[2 * i] = p->L + i * w;
        I[2 * i + 1] = p->L + (i + 1) * w;
        n_pieces[i] = 0;
    }
    // the guided portion of group i is the cumulative range [i G/N, (i+1) G/N)
    for (int j = 0; j < pl.jstar; ++j) {
        const double lo = p->h_wlo[j], hi = std::min(p->h_whi[j], pl.Ubar), c0 = p->h_wcum[j];
        for (int i = 0; i < N; ++i) {
            const double a = std::max(pl.G * i / N, c0), b = std::min(pl.G * (i + 1) / N, c0 + (hi - lo));
            if (b > a && n_pieces[i] < maxp) {
                pieces[((size_t)i * maxp + n_pieces[i]) * 2] = lo + (a - c0);
                pieces[((size_t)i * maxp + n_pieces[i]) * 2 + 1] = lo + (b - c0);
                n_pieces[i]++;
            }
        }
    }
    return ST_OK;
}

}  // extern "C"
