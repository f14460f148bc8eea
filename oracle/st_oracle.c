/*
 * st_oracle.c -- FP64 CPU oracle for the ST-pRRTC space-time extend path.
 *
 * TEST INFRASTRUCTURE ONLY (see st_oracle.h).  Plain, scalar, double
 * precision, single-threaded; no blocking, fusion or reordering beyond what
 * the paper's definitions state.  Node numbering is a data convention shared
 * with the device path through exported snapshots: pool 0 is the forward
 * tree, pool 1+i is backward group i (interval root) or slot i (root
 * recycling); inside a pool nodes are numbered in insertion order, and the
 * global index is base(pool) + local index with base(0) = 0 and
 * base(1+i) = cap_fwd + i * cap_bwd.
 */
#include "st_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define INF (1.0 / 0.0)
#define PI 3.14159265358979323846

/* ========================================================================= */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Each round        */
/* multiplies words 0 and 2 by fixed odd constants, swaps the halves and     */
/* mixes in the key; the key is bumped by the Weyl constants between rounds. */
/* ========================================================================= */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

/* A 32-bit draw mapped to [0,1): the top 24 bits times 2^-24.  The value is
 * exactly representable in single precision, so both sides see the same
 * number. */
static double unit24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* Uniform index in {0..n-1} from a draw, in integer arithmetic. */
static int32_t index24(uint32_t x, int32_t n) { return (int32_t)(((uint64_t)(x >> 8) * (uint64_t)n) >> 24); }

/* The draws of one worker in one iteration: Philox blocks keyed by (seed,
 * problem) with counter (iteration, worker, block, 0); four blocks for the
 * plain sampler, seven with the learned proposal. */
static void worker_draws(const orc_scene *sc, int64_t iter, int64_t w, uint32_t u[28], int nblk) {
    uint32_t key[2] = {sc->seed, sc->problem_id};
    for (uint32_t b = 0; b < (uint32_t)nblk; ++b) {
        uint32_t ctr[4] = {(uint32_t)iter, (uint32_t)w, b, 0u};
        orc_philox4x32_10(ctr, key, u + 4 * b);
    }
}

/* ========================================================================= */
/* Geometry: robot spheres (standard DH chain) and obstacle motion.          */
/* ========================================================================= */

typedef struct { double m[4][4]; } mat4;

static mat4 mat_identity(void) {
    mat4 r;
    memset(&r, 0, sizeof r);
    for (int i = 0; i < 4; ++i) r.m[i][i] = 1.0;
    return r;
}

static mat4 mat_mul(const mat4 *a, const mat4 *b) {
    mat4 r;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += a->m[i][k] * b->m[k][j];
            r.m[i][j] = s;
        }
    return r;
}

static mat4 rot_z(double th) {
    mat4 r = mat_identity();
    r.m[0][0] = cos(th); r.m[0][1] = -sin(th);
    r.m[1][0] = sin(th); r.m[1][1] = cos(th);
    return r;
}

static mat4 rot_x(double al) {
    mat4 r = mat_identity();
    r.m[1][1] = cos(al); r.m[1][2] = -sin(al);
    r.m[2][1] = sin(al); r.m[2][2] = cos(al);
    return r;
}

static mat4 trans(double x, double y, double z) {
    mat4 r = mat_identity();
    r.m[0][3] = x; r.m[1][3] = y; r.m[2][3] = z;
    return r;
}

/* Frames T_0 = I, T_i = T_{i-1} Rz(q_i + theta0_i) Tz(d_i) Tx(a_i) Rx(alpha_i).
 * frames_out: (d+1) x 12 row-major 3x4 blocks. */
void orc_frames(const orc_scene *sc, const double *q, double *frames_out) {
    mat4 T = mat_identity();
    for (int i = 0; i <= sc->d; ++i) {
        if (i > 0) {
            const double *p = sc->dh[i - 1];
            mat4 A = rot_z(q[i - 1] + p[3]);
            mat4 B = trans(0.0, 0.0, p[2]);
            mat4 C = trans(p[0], 0.0, 0.0);
            mat4 D = rot_x(p[1]);
            mat4 t1 = mat_mul(&T, &A);
            mat4 t2 = mat_mul(&t1, &B);
            mat4 t3 = mat_mul(&t2, &C);
            T = mat_mul(&t3, &D);
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 4; ++c) frames_out[i * 12 + r * 4 + c] = T.m[r][c];
    }
}

/* Sphere centres in the world frame, out: S x 3. */
void orc_sphere_centres(const orc_scene *sc, const double *q, double *out) {
    if (sc->kind == ORC_KIND_TRANSLATE) {
        for (int s = 0; s < sc->n_sph; ++s) {
            out[3 * s + 0] = q[0] + sc->sph[s][0];
            out[3 * s + 1] = q[1] + sc->sph[s][1];
            out[3 * s + 2] = (sc->d >= 3 ? q[2] : 0.0) + sc->sph[s][2];
        }
        return;
    }
    double frames[(ORC_MAX_DOF + 1) * 12];
    orc_frames(sc, q, frames);
    for (int s = 0; s < sc->n_sph; ++s) {
        const double *F = frames + 12 * sc->sph_link[s];
        for (int r = 0; r < 3; ++r)
            out[3 * s + r] = F[r * 4 + 0] * sc->sph[s][0] + F[r * 4 + 1] * sc->sph[s][1] +
                             F[r * 4 + 2] * sc->sph[s][2] + F[r * 4 + 3];
    }
}

/* Obstacle centre at absolute time t: linear interpolation between the
 * waypoints that bracket t, held at the first/last waypoint outside their
 * time span (obstacles are interpolated at each query time, Sec. VI). */
void orc_obstacle_pos(const orc_scene *sc, int o, double t, double *out) {
    int n = sc->n_wp[o];
    const double (*w)[4] = sc->wp[o];
    if (n == 1 || t <= w[0][0]) {
        out[0] = w[0][1]; out[1] = w[0][2]; out[2] = w[0][3];
        return;
    }
    if (t >= w[n - 1][0]) {
        out[0] = w[n - 1][1]; out[1] = w[n - 1][2]; out[2] = w[n - 1][3];
        return;
    }
    int k = 0;
    while (k + 1 < n - 1 && w[k + 1][0] <= t) ++k;
    double span = w[k + 1][0] - w[k][0];
    double s = span > 0.0 ? (t - w[k][0]) / span : 0.0;
    for (int c = 0; c < 3; ++c) out[c] = w[k][1 + c] + s * (w[k + 1][1 + c] - w[k][1 + c]);
}

/* ========================================================================= */
/* State and edge validity.                                                  */
/* ========================================================================= */

/* Distance from point c to a closed oriented box: in the box's axes the
 * offset u_a = axis_a . (c - centre); the excess over the half extent,
 * max(|u_a| - h_a, 0), is the offset to the nearest box point along that
 * axis, so the distance is the norm of the three excesses (0 inside). */
static double box_distance(const double *B, const double *c) {
    double e2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double *ax = B + 6 + 3 * a;
        double u = ax[0] * (c[0] - B[0]) + ax[1] * (c[1] - B[1]) + ax[2] * (c[2] - B[2]);
        double ex = fabs(u) - B[3 + a];
        if (ex > 0.0) e2 += ex * ex;
    }
    return sqrt(e2);
}

/* valid(q,t) <=> q in C, 0 <= t <= H, and every robot sphere / obstacle pair
 * is at least r_s + r_o apart (touching counts as free; Eq. 1 with the
 * sphere model).  With static geometry, also every robot sphere is at least
 * its radius from every box, and every sphere pair of a listed link pair is
 * at least r_s + r_s' apart.  margin receives the least signed clearance over
 * all these pairs, and the distance to the box bounds. */
int orc_state_valid(const orc_scene *sc, const double *x, double *margin) {
    int d = sc->d;
    double t = x[d];
    double m = INF;
    int ok = 1;
    for (int j = 0; j < d; ++j) {
        double b = fmin(x[j] - sc->q_lo[j], sc->q_hi[j] - x[j]);
        if (b < 0.0) ok = 0;
        m = fmin(m, b);
    }
    /* the time bounds enter the margin only when violated: the forward root
     * sits exactly at t = 0 and is not a numerical hazard */
    double bt = fmin(t, sc->t_max - t);
    if (bt < 0.0) {
        ok = 0;
        m = fmin(m, bt);
    }
    double cs[ORC_MAX_SPH * 3];
    orc_sphere_centres(sc, x, cs);
    for (int o = 0; o < sc->n_obs; ++o) {
        double co[3];
        orc_obstacle_pos(sc, o, t, co);
        for (int s = 0; s < sc->n_sph; ++s) {
            double dx = cs[3 * s] - co[0], dy = cs[3 * s + 1] - co[1], dz = cs[3 * s + 2] - co[2];
            double dist = sqrt(dx * dx + dy * dy + dz * dz);
            double R = sc->sph[s][3] + sc->obs_r[o];
            if (dist < R) ok = 0;
            m = fmin(m, dist - R);
        }
    }
    for (int b = 0; b < sc->n_box; ++b)
        for (int s = 0; s < sc->n_sph; ++s) {
            double dist = box_distance(sc->box[b], cs + 3 * s);
            double R = sc->sph[s][3];
            if (dist < R) ok = 0;
            m = fmin(m, dist - R);
        }
    for (int k = 0; k < sc->n_self; ++k) {
        int la = sc->self_pair[k][0], lb = sc->self_pair[k][1];
        for (int s = 0; s < sc->n_sph; ++s) {
            if (sc->sph_link[s] != la) continue;
            for (int u = 0; u < sc->n_sph; ++u) {
                if (sc->sph_link[u] != lb) continue;
                double dx = cs[3 * s] - cs[3 * u], dy = cs[3 * s + 1] - cs[3 * u + 1], dz = cs[3 * s + 2] - cs[3 * u + 2];
                double dist = sqrt(dx * dx + dy * dy + dz * dz);
                double R = sc->sph[s][3] + sc->sph[u][3];
                if (dist < R) ok = 0;
                m = fmin(m, dist - R);
            }
        }
    }
    if (margin) *margin = m;
    return ok;
}

/* Discretised edge validity.  Reading (the paper only says edges are checked
 * along their interpolation at absolute times): order the endpoints by time,
 * take n = max(1, ceil(max(D, v_max (t_b - t_a)) / h)) steps and check the
 * n+1 states q_a + (j/n)(q_b - q_a), t_a + (j/n)(t_b - t_a).  first_hit is
 * the least colliding j in that order, or -1.  min_abs_margin is the least
 * |margin| over the states a first-hit checker must look at (all states of a
 * free edge, states 0..first_hit otherwise).  n_real = max(D, v dt) / h. */
int orc_edge_check(const orc_scene *sc, const double *xa_in, const double *xb_in, int32_t *first_hit,
                   int64_t *n_states, double *min_abs_margin, double *n_real) {
    int d = sc->d;
    const double *xa = xa_in, *xb = xb_in;
    if (xa[d] > xb[d]) { const double *tmp = xa; xa = xb; xb = tmp; }
    double D2 = 0.0;
    for (int j = 0; j < d; ++j) D2 += (xb[j] - xa[j]) * (xb[j] - xa[j]);
    double D = sqrt(D2);
    double span = fmax(D, sc->v_max * (xb[d] - xa[d]));
    double nr = span / sc->h;
    int64_t n = (int64_t)ceil(nr);
    if (n < 1) n = 1;
    int32_t hit = -1;
    double mabs = INF;
    double x[ORC_MAX_DOF + 1];
    for (int64_t j = 0; j <= n; ++j) {
        double s = (double)j / (double)n;
        /* s = 1 is the endpoint itself */
        for (int c = 0; c <= d; ++c) x[c] = j == n ? xb[c] : xa[c] + s * (xb[c] - xa[c]);
        double m;
        int ok = orc_state_valid(sc, x, &m);
        mabs = fmin(mabs, fabs(m));
        if (!ok) { hit = (int32_t)j; break; }
    }
    if (first_hit) *first_hit = hit;
    if (n_states) *n_states = n;
    if (min_abs_margin) *min_abs_margin = mabs;
    if (n_real) *n_real = nr;
    return hit < 0;
}

void orc_check_edges(const orc_scene *sc, int64_t E, const double *xa, const double *xb, uint8_t *free_out,
                     int32_t *first_hit, int64_t *n_states, double *min_abs_margin, double *n_real) {
    int w = sc->d + 1;
    for (int64_t e = 0; e < E; ++e)
        free_out[e] = (uint8_t)orc_edge_check(sc, xa + e * w, xb + e * w, first_hit ? first_hit + e : NULL,
                                              n_states ? n_states + e : NULL,
                                              min_abs_margin ? min_abs_margin + e : NULL, n_real ? n_real + e : NULL);
}

void orc_check_states(const orc_scene *sc, int64_t M, const double *x, uint8_t *free_out, double *margin) {
    int w = sc->d + 1;
    for (int64_t i = 0; i < M; ++i) free_out[i] = (uint8_t)orc_state_valid(sc, x + i * w, margin ? margin + i : NULL);
}

/* Exact continuous check for a translating disc/sphere robot with one sphere
 * against obstacles on a single constant-velocity segment over the edge's time
 * span: the relative position p(tau) = p0 + w tau is linear, its closest
 * approach is at tau* = clamp(-p0.w / |w|^2, 0, T).  Returns 1 when every
 * pair stays at distance >= R, and the least (distance - R) in dmin.  Only
 * the moving obstacles enter (static boxes and link pairs belong to arms). */
int orc_edge_continuous(const orc_scene *sc, const double *xa_in, const double *xb_in, double *dmin) {
    int d = sc->d;
    const double *xa = xa_in, *xb = xb_in;
    if (xa[d] > xb[d]) { const double *tmp = xa; xa = xb; xb = tmp; }
    double T = xb[d] - xa[d];
    double best = INF;
    for (int o = 0; o < sc->n_obs; ++o) {
        double c0[3], c1[3];
        orc_obstacle_pos(sc, o, xa[d], c0);
        orc_obstacle_pos(sc, o, xb[d], c1);
        for (int s = 0; s < sc->n_sph; ++s) {
            double ra[3] = {xa[0] + sc->sph[s][0], xa[1] + sc->sph[s][1], (d >= 3 ? xa[2] : 0.0) + sc->sph[s][2]};
            double rb[3] = {xb[0] + sc->sph[s][0], xb[1] + sc->sph[s][1], (d >= 3 ? xb[2] : 0.0) + sc->sph[s][2]};
            double p0[3], w[3];
            for (int c = 0; c < 3; ++c) {
                p0[c] = ra[c] - c0[c];
                w[c] = T > 0.0 ? ((rb[c] - ra[c]) - (c1[c] - c0[c])) / T : 0.0;
            }
            double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
            double tau = 0.0;
            if (ww > 0.0) {
                tau = -(p0[0] * w[0] + p0[1] * w[1] + p0[2] * w[2]) / ww;
                if (tau < 0.0) tau = 0.0;
                if (tau > T) tau = T;
            }
            double dist = 0.0;
            for (int c = 0; c < 3; ++c) dist += (p0[c] + w[c] * tau) * (p0[c] + w[c] * tau);
            dist = sqrt(dist) - (sc->sph[s][3] + sc->obs_r[o]);
            if (dist < best) best = dist;
        }
    }
    if (dmin) *dmin = best;
    return best >= 0.0;
}

/* Exact continuous check of an edge for a translating robot against
 * obstacles on piecewise-linear trajectories: the edge's time span is cut at
 * every waypoint time of the obstacle strictly inside it; on each piece both
 * the robot (linear along the edge) and the obstacle (one constant-velocity
 * segment, or held) move linearly, so each sphere pair's relative position is
 * affine in time and its closest approach has the closed form
 * u* = clamp(-p0.(p1-p0) / |p1-p0|^2, 0, 1) between the piece's end values.
 * The box and horizon hold along the edge iff they hold at both endpoints
 * (convex sets).  Free iff they hold and every pair keeps distance >= R
 * (touching is free); dmin receives the least pair clearance.  Only the
 * moving obstacles enter (static boxes and link pairs belong to arms). */
int orc_edge_continuous_pw(const orc_scene *sc, const double *xa_in, const double *xb_in, double *dmin) {
    const int d = sc->d;
    const double *xa = xa_in, *xb = xb_in;
    if (xa[d] > xb[d]) { const double *tmp = xa; xa = xb; xb = tmp; }
    int ok = 1;
    for (int e = 0; e < 2; ++e) {
        const double *x = e ? xb : xa;
        if (!(x[d] >= 0.0) || !(x[d] <= sc->t_max)) ok = 0;
        for (int j = 0; j < d; ++j)
            if (!(x[j] >= sc->q_lo[j]) || !(x[j] <= sc->q_hi[j])) ok = 0;
    }
    const double ta = xa[d], tb = xb[d], T = tb - ta;
    double best = INF;
    for (int o = 0; o < sc->n_obs; ++o) {
        /* piece boundaries: ta, the waypoint times strictly inside, tb */
        double cut[ORC_MAX_WP + 2];
        int nc = 0;
        cut[nc++] = ta;
        for (int k = 0; k < sc->n_wp[o]; ++k)
            if (sc->wp[o][k][0] > ta && sc->wp[o][k][0] < tb) cut[nc++] = sc->wp[o][k][0];
        cut[nc++] = tb;
        for (int pc = 0; pc + 1 < nc; ++pc) {
            const double t0 = cut[pc], t1 = cut[pc + 1];
            double c0[3], c1[3], q0[3] = {0, 0, 0}, q1[3] = {0, 0, 0};
            orc_obstacle_pos(sc, o, t0, c0);
            orc_obstacle_pos(sc, o, t1, c1);
            const double f0 = T > 0.0 ? (t0 - ta) / T : 0.0, f1 = T > 0.0 ? (t1 - ta) / T : 0.0;
            for (int j = 0; j < d && j < 3; ++j) {
                q0[j] = xa[j] + f0 * (xb[j] - xa[j]);
                q1[j] = xa[j] + f1 * (xb[j] - xa[j]);
            }
            for (int s = 0; s < sc->n_sph; ++s) {
                double p0[3], dp[3], pp = 0.0, pd = 0.0;
                for (int c = 0; c < 3; ++c) {
                    p0[c] = q0[c] + sc->sph[s][c] - c0[c];
                    dp[c] = (q1[c] + sc->sph[s][c] - c1[c]) - p0[c];
                    pp += dp[c] * dp[c];
                    pd += p0[c] * dp[c];
                }
                double u = 0.0;
                if (pp > 0.0) {
                    u = -pd / pp;
                    if (u < 0.0) u = 0.0;
                    if (u > 1.0) u = 1.0;
                }
                double dist = 0.0;
                for (int c = 0; c < 3; ++c) dist += (p0[c] + u * dp[c]) * (p0[c] + u * dp[c]);
                dist = sqrt(dist) - (sc->sph[s][3] + sc->obs_r[o]);
                if (dist < best) best = dist;
            }
        }
    }
    if (dmin) *dmin = best;
    return ok && best >= 0.0;
}

/* ========================================================================= */
/* Directed space-time distance (Eq. 7) and nearest-node search (Alg. 1).   */
/* ========================================================================= */

static double config_dist(int d, const double *a, const double *b) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) s += (b[j] - a[j]) * (b[j] - a[j]);
    return sqrt(s);
}

/* rho_sigma(x, x_r): infinite unless Delta = sigma (t_r - t) > 0 and
 * D(q, q_r) <= v Delta; otherwise sqrt((D^2 + v^2 (t_r - t)^2) / 2). */
double orc_rho(int d, double v, int sigma, const double *x, const double *xr) {
    double D = config_dist(d, x, xr);
    double delta = sigma * (xr[d] - x[d]);
    if (!(delta > 0.0) || !(D <= v * delta)) return INF;
    double dt = xr[d] - x[d];
    return sqrt((D * D + v * v * dt * dt) / 2.0);
}

/* Nearest node over nodes[0..n) (rows of d+1, time last) restricted to
 * mask[i] != 0 (mask may be NULL).  metric RHO uses Eq. 7; CONFIG uses the
 * configuration distance D (root recycling).  Lowest index wins ties (the
 * paper does not say).  Returns -1 with dist = +inf when nothing qualifies.
 * amb (optional) is set when the choice is numerically fragile: a runner-up
 * within a relative 1e-5 of the best, or (RHO) a node within 1e-5 of the
 * speed cone whose unconstrained distance is within 1e-5 of the best. */
int64_t orc_nearest(const orc_scene *sc, int64_t n, const double *nodes, const uint8_t *mask, int sigma,
                    int metric, const double *xq, double *dist, uint8_t *amb) {
    int d = sc->d, w = d + 1;
    double v = sc->v_max;
    int64_t best = -1;
    double bd = INF;
    for (int64_t i = 0; i < n; ++i) {
        if (mask && !mask[i]) continue;
        const double *x = nodes + i * w;
        double r = metric == ORC_METRIC_RHO ? orc_rho(d, v, sigma, x, xq) : config_dist(d, x, xq);
        if (r < bd) { bd = r; best = i; }
    }
    if (dist) *dist = bd;
    if (amb) {
        uint8_t a = 0;
        double lim = isinf(bd) ? INF : bd * (1.0 + 1e-5) + 1e-12;
        for (int64_t i = 0; i < n && !a; ++i) {
            if (mask && !mask[i]) continue;
            if (i == best) continue;
            const double *x = nodes + i * w;
            if (metric == ORC_METRIC_RHO) {
                double D = config_dist(d, x, xq);
                double del = sigma * (xq[d] - x[d]);
                double vd = v * del;
                double raw = sqrt((D * D + v * v * (xq[d] - x[d]) * (xq[d] - x[d])) / 2.0);
                double r = orc_rho(d, v, sigma, x, xq);
                if (r <= lim) a = 1;
                if (del > 0.0 && fabs(D * D - vd * vd) <= 1e-5 * vd * vd && raw <= lim) a = 1;
            } else {
                if (config_dist(d, x, xq) <= lim) a = 1;
            }
        }
        *amb = a;
    }
    return best;
}

/* ========================================================================= */
/* Goal grid, guided windows and the interval-root partition (Sec. IV-B).    */
/* ========================================================================= */

/* Lower bound L_g = D(q_s, q_g) / v_max (Eq. 5).  With the arrival range
 * [t_min, t_max] of the problem the search domain is [L, H] with
 * L = max(L_g, t_min) and H = t_max (reading: the paper's domain is [L_g, H]). */
double orc_lower_bound(const orc_scene *sc) {
    double Lg = config_dist(sc->d, sc->q_s, sc->q_g) / sc->v_max;
    return fmax(Lg, sc->t_min);
}

/* Grid indices k with k dt in [L, H]: k_lo = ceil(L/dt), k_hi = floor(H/dt)
 * (Eq. 5's first reachable index).  free_out[k - k_lo] = valid(q_g, k dt). */
void orc_goal_grid_range(const orc_scene *sc, int64_t *k_lo, int64_t *k_hi) {
    double L = orc_lower_bound(sc);
    *k_lo = (int64_t)ceil(L / sc->dt);
    *k_hi = (int64_t)floor(sc->t_max / sc->dt);
}

void orc_goal_grid(const orc_scene *sc, int64_t k_lo, int64_t k_hi, uint8_t *free_out) {
    double x[ORC_MAX_DOF + 1];
    for (int j = 0; j < sc->d; ++j) x[j] = sc->q_g[j];
    for (int64_t k = k_lo; k <= k_hi; ++k) {
        x[sc->d] = (double)k * sc->dt;
        free_out[k - k_lo] = (uint8_t)orc_state_valid(sc, x, NULL);
    }
}

/* Interval-root allocation for Ubar = min(H, U):
 *  - each free check k gives the window [k dt - dt/2, k dt + dt/2] clipped to
 *    [L, H]; touching windows merge into guided windows;
 *  - uniform intervals I_i = [L + i w, L + (i+1) w), w = (Ubar - L) / N;
 *  - the guided windows clipped to [L, Ubar) have total length G; walking them
 *    in time order, group i receives the portions between cumulative lengths
 *    i G / N and (i+1) G / N (gaps between windows are skipped).
 * Outputs: I (N x 2), n_pieces (N), pieces (N x maxp x 2).  Returns the total
 * number of pieces, or -1 if some group needs more than maxp pieces. */
int orc_ir_partition(double L, double H, double Ubar, double dt, int64_t k_lo, int64_t k_hi, const uint8_t *free_k,
                     int N, double *I, int32_t *n_pieces, double *pieces, int maxp) {
    double w = (Ubar - L) / N;
    for (int i = 0; i < N; ++i) {
        I[2 * i] = L + i * w;
        I[2 * i + 1] = L + (i + 1) * w;
        n_pieces[i] = 0;
    }
    /* merged windows, clipped to [L, H] then to [L, Ubar) */
    int64_t nk = k_hi - k_lo + 1;
    double *wl = (double *)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    double *wh = (double *)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    int64_t nw = 0;
    for (int64_t k = k_lo; k <= k_hi; ++k) {
        if (!free_k[k - k_lo]) continue;
        int64_t k2 = k;
        while (k2 + 1 <= k_hi && free_k[k2 + 1 - k_lo]) ++k2;
        double lo = fmax(k * dt - dt / 2.0, L);
        double hi = fmin(k2 * dt + dt / 2.0, H);
        lo = fmax(lo, L);
        hi = fmin(hi, Ubar);
        if (hi > lo) { wl[nw] = lo; wh[nw] = hi; ++nw; }
        k = k2;
    }
    double G = 0.0;
    for (int64_t j = 0; j < nw; ++j) G += wh[j] - wl[j];
    int total = 0, ok = 1;
    if (G > 0.0) {
        double cum = 0.0;
        for (int64_t j = 0; j < nw; ++j) {
            double len = wh[j] - wl[j];
            for (int i = 0; i < N; ++i) {
                double c0 = G * i / N, c1 = G * (i + 1) / N;
                double a = fmax(c0, cum), b = fmin(c1, cum + len);
                if (b > a) {
                    if (n_pieces[i] >= maxp) { ok = 0; continue; }
                    double *p = pieces + ((size_t)i * maxp + n_pieces[i]) * 2;
                    p[0] = wl[j] + (a - cum);
                    p[1] = wl[j] + (b - cum);
                    n_pieces[i]++;
                    total++;
                }
            }
            cum += len;
        }
    }
    free(wl);
    free(wh);
    return ok ? total : -1;
}

/* ========================================================================= */
/* Planner state.                                                            */
/* ========================================================================= */

#define ORC_MAXP 4096

struct orc_planner {
    orc_scene sc;
    int n_pools;
    int64_t base[1 + 256], cap[1 + 256], count[1 + 256];
    int64_t total;
    double *x;        /* total x (d+1): configuration then time */
    double *cost;     /* path length to the tree root */
    double *rootT;    /* root time of the node's tree (backward), 0 for forward */
    int32_t *parent;  /* global index, -1 for a root */
    /* incumbent */
    double U, C;
    int64_t inc_f, inc_b;
    int64_t first_iter;
    /* domain and goal grid */
    double L, H;
    int64_t k_lo, k_hi;
    uint8_t *gfree;
    /* interval root */
    double I[256 * 2];
    int32_t np[256];
    double *pieces; /* N x ORC_MAXP x 2 */
    /* root recycling */
    double slotT[256];
    int64_t slotK[256];
    int32_t slot_active[256];
    uint32_t slot_gen[256];
    int32_t n_active;
    int32_t active_list[256];
    int64_t iter;
    int32_t overflow;
    int64_t n_edge_checks, n_bridge_checks; /* edges decided (for throughput) */
    /* learned proposal (an addition to the paper's method) */
    double prop_mix, prop_wcum[8], prop_mu[64], prop_sd[64], prop_hcum[32];
};

/* Install the proposal network's output z[168] (8 mixture logits, 8x8 means,
 * 8x8 log standard deviations of the normalised state q/pi, t/60; 32
 * arrival-histogram logits over [t_min, t_max]) and the probability mix of a
 * learned draw.  z = NULL or mix = 0 switches the proposal off. */
void orc_planner_set_proposal(orc_planner *p, const double *z, double mix) {
    p->prop_mix = 0.0;
    if (!z || !(mix > 0.0)) return;
    double mx = -INF, s = 0.0, acc = 0.0;
    for (int c = 0; c < 8; ++c) mx = fmax(mx, z[c]);
    for (int c = 0; c < 8; ++c) s += exp(z[c] - mx);
    for (int c = 0; c < 8; ++c) {
        acc += exp(z[c] - mx) / s;
        p->prop_wcum[c] = acc;
    }
    p->prop_wcum[7] = 1.0;
    for (int i = 0; i < 64; ++i) {
        p->prop_mu[i] = z[8 + i];
        p->prop_sd[i] = exp(z[72 + i]);
    }
    mx = -INF;
    s = 0.0;
    acc = 0.0;
    for (int b = 0; b < 32; ++b) mx = fmax(mx, z[136 + b]);
    for (int b = 0; b < 32; ++b) s += exp(z[136 + b] - mx);
    for (int b = 0; b < 32; ++b) {
        acc += exp(z[136 + b] - mx) / s;
        p->prop_hcum[b] = acc;
    }
    p->prop_hcum[31] = 1.0;
    p->prop_mix = mix;
}

static int64_t push_node(orc_planner *p, int pool, const double *x, int32_t parent, double cost, double rootT) {
    if (p->count[pool] >= p->cap[pool]) { p->overflow = 1; return -1; }
    int64_t idx = p->base[pool] + p->count[pool]++;
    int w = p->sc.d + 1;
    memcpy(p->x + idx * w, x, sizeof(double) * (size_t)w);
    p->parent[idx] = parent;
    p->cost[idx] = cost;
    p->rootT[idx] = rootT;
    return idx;
}

static void ir_repartition(orc_planner *p) {
    double Ubar = fmin(p->H, p->U);
    int N = p->sc.n_groups;
    if (!(p->L < Ubar)) return;
    orc_ir_partition(p->L, p->H, Ubar, p->sc.dt, p->k_lo, p->k_hi, p->gfree, N, p->I, p->np, p->pieces, ORC_MAXP);
}

static void rr_refresh_active(orc_planner *p) {
    p->n_active = 0;
    for (int i = 0; i < p->sc.n_groups; ++i)
        if (p->slot_active[i]) p->active_list[p->n_active++] = i;
}

static double grid_time(const orc_planner *p, int64_t k) { return (double)k * p->sc.dt; }

/* Reading of "choose up to N collision-free roots in [L_grid, H)": split the
 * grid indices k_lo..k_end-1 (k dt < H) into N equal integer strata; slot j
 * takes the first free grid time of stratum j, or stays empty (inactive). */
static void rr_init_roots(orc_planner *p) {
    int N = p->sc.n_groups;
    int64_t k_end = p->k_hi + 1;
    while (k_end > p->k_lo && grid_time(p, k_end - 1) >= p->H) --k_end;
    int64_t K = k_end - p->k_lo;
    double xg[ORC_MAX_DOF + 1];
    for (int j = 0; j < p->sc.d; ++j) xg[j] = p->sc.q_g[j];
    for (int s = 0; s < N; ++s) {
        p->slot_active[s] = 0;
        p->slotT[s] = INF;
        p->slotK[s] = -1;
        p->slot_gen[s] = 0;
        if (K <= 0) continue;
        int64_t a = p->k_lo + (K * s) / N, b = p->k_lo + (K * (s + 1)) / N;
        for (int64_t k = a; k < b; ++k) {
            if (!p->gfree[k - p->k_lo]) continue;
            xg[p->sc.d] = grid_time(p, k);
            p->slotT[s] = xg[p->sc.d];
            p->slotK[s] = k;
            p->slot_active[s] = 1;
            push_node(p, 1 + s, xg, -1, 0.0, xg[p->sc.d]);
            break;
        }
    }
    rr_refresh_active(p);
}

/* Root recycling after a strict drop of U (Sec. V, Alg. 3): roots with
 * T_i >= U become inactive; slots with T_i > U are donors.  Reading of the
 * replacement search: split the grid indices below U (k dt < U) into N equal
 * strata; walking the strata that hold no retained active root in time order,
 * each gives its first free grid time to the next donor (slot order).  A
 * donor that receives a root discards its tree (generation + 1) and gets the
 * empty root; a donor without one stays inactive.  The no-recycling ablation
 * of the evaluation (Sec. VI) keeps the initial roots: deactivation only. */
static void rr_update(orc_planner *p) {
    int N = p->sc.n_groups;
    double U = p->U;
    int donors[256], nd = 0;
    for (int s = 0; s < N; ++s) {
        if (p->slotT[s] >= U) p->slot_active[s] = 0;
        if (p->slotT[s] > U) donors[nd++] = s;
    }
    int64_t k_end = p->k_lo;
    while (k_end <= p->k_hi && grid_time(p, k_end) < U) ++k_end;
    int64_t K = k_end - p->k_lo;
    if (p->sc.no_recycling) K = 0;
    int di = 0;
    double xg[ORC_MAX_DOF + 1];
    for (int j = 0; j < p->sc.d; ++j) xg[j] = p->sc.q_g[j];
    for (int st = 0; st < N && di < nd && K > 0; ++st) {
        int64_t a = p->k_lo + (K * st) / N, b = p->k_lo + (K * (st + 1)) / N;
        int occupied = 0;
        for (int s = 0; s < N; ++s)
            if (p->slot_active[s] && p->slotK[s] >= a && p->slotK[s] < b) occupied = 1;
        if (occupied) continue;
        for (int64_t k = a; k < b; ++k) {
            if (!p->gfree[k - p->k_lo]) continue;
            int s = donors[di++];
            p->slot_gen[s]++;
            p->count[1 + s] = 0;
            xg[p->sc.d] = grid_time(p, k);
            p->slotT[s] = xg[p->sc.d];
            p->slotK[s] = k;
            p->slot_active[s] = 1;
            push_node(p, 1 + s, xg, -1, 0.0, xg[p->sc.d]);
            break;
        }
    }
    rr_refresh_active(p);
}

orc_planner *orc_planner_create(const orc_scene *sc) {
    orc_planner *p = (orc_planner *)calloc(1, sizeof(orc_planner));
    p->sc = *sc;
    int N = sc->n_groups;
    p->n_pools = 1 + N;
    p->base[0] = 0;
    p->cap[0] = sc->cap_fwd;
    for (int i = 0; i < N; ++i) {
        p->base[1 + i] = (int64_t)sc->cap_fwd + (int64_t)i * sc->cap_bwd;
        p->cap[1 + i] = sc->cap_bwd;
    }
    p->total = (int64_t)sc->cap_fwd + (int64_t)N * sc->cap_bwd;
    int w = sc->d + 1;
    p->x = (double *)calloc((size_t)(p->total * w), sizeof(double));
    p->cost = (double *)calloc((size_t)p->total, sizeof(double));
    p->rootT = (double *)calloc((size_t)p->total, sizeof(double));
    p->parent = (int32_t *)calloc((size_t)p->total, sizeof(int32_t));
    p->pieces = (double *)calloc((size_t)N * ORC_MAXP * 2, sizeof(double));
    p->U = INF;
    p->C = INF;
    p->inc_f = p->inc_b = -1;
    p->first_iter = -1;
    p->L = orc_lower_bound(sc);
    p->H = sc->t_max;
    orc_goal_grid_range(sc, &p->k_lo, &p->k_hi);
    int64_t nk = p->k_hi - p->k_lo + 1;
    p->gfree = (uint8_t *)calloc((size_t)(nk > 0 ? nk : 1), 1);
    if (nk > 0) orc_goal_grid(sc, p->k_lo, p->k_hi, p->gfree);
    double xs[ORC_MAX_DOF + 1];
    for (int j = 0; j < sc->d; ++j) xs[j] = sc->q_s[j];
    xs[sc->d] = 0.0;
    push_node(p, 0, xs, -1, 0.0, 0.0);
    if (sc->variant == ORC_IR)
        ir_repartition(p);
    else
        rr_init_roots(p);
    return p;
}

void orc_planner_destroy(orc_planner *p) {
    if (!p) return;
    free(p->x); free(p->cost); free(p->rootT); free(p->parent); free(p->gfree); free(p->pieces);
    free(p);
}

/* Does backward group g own a tree rooted below U?  (IR: trees rooted at
 * T >= U are inactive.) */
static int ir_group_active(const orc_planner *p, int g) {
    int pool = 1 + g;
    for (int64_t i = 0; i < p->count[pool]; ++i) {
        int64_t idx = p->base[pool] + i;
        if (p->parent[idx] < 0 && p->rootT[idx] < p->U) return 1;
    }
    return 0;
}

/* ========================================================================= */
/* Sampling (Sec. IV-B with Eq. 6 for interval root; Alg. 3 for recycling). */
/* Draws: u[0] group, u[1] guided-vs-uniform, u[2] piece, u[3] position,     */
/* u[4..10] q_r, u[11] t_r, u[12] p_new; learned proposal: u[13] learned or  */
/* plain, u[14] component, u[15] histogram bin, u[16..23] Box-Muller pairs,  */
/* u[24] position inside the bin.                                            */
/* Reading: direction alternates as (worker + iteration) mod 2, 0 = forward. */
/* ========================================================================= */

void orc_planner_sample(orc_planner *p, int64_t iter, int64_t B, int8_t *dir, uint8_t *flags, int32_t *grp,
                        double *T, double *qr /* d x B */, double *tr) {
    const orc_scene *sc = &p->sc;
    int d = sc->d, N = sc->n_groups;
    double v = sc->v_max;
    double Ubar = fmin(p->H, p->U);
    uint8_t gact[256];
    if (sc->variant == ORC_IR)
        for (int g = 0; g < N; ++g) gact[g] = (uint8_t)ir_group_active(p, g);
    for (int64_t w = 0; w < B; ++w) {
        uint32_t u[28];
        const int learned = p->prop_mix > 0.0;
        worker_draws(sc, iter, w, u, learned ? 7 : 4);
        int8_t dr = (int8_t)((w + iter) & 1);
        uint8_t fl = 0;
        int32_t g = 0;
        double Tw = 0.0, trw = 0.0;
        double q[ORC_MAX_DOF];
        for (int j = 0; j < d; ++j) q[j] = sc->q_lo[j] + unit24(u[4 + j]) * (sc->q_hi[j] - sc->q_lo[j]);
        /* learned draw: (q, t) from the mixture component chosen by u[14],
         * Gaussian variates by the Box-Muller transform */
        const int use_net = learned && unit24(u[13]) < p->prop_mix;
        double ylearn_t = 0.0;
        if (use_net) {
            fl |= ORC_LEARNED;
            int c = 0;
            while (c < 7 && !(unit24(u[14]) < p->prop_wcum[c])) ++c;
            double nrm[8];
            for (int k = 0; k < 4; ++k) {
                double r = sqrt(-2.0 * log(1.0 - unit24(u[16 + 2 * k])));
                double th = 2.0 * PI * unit24(u[17 + 2 * k]);
                nrm[2 * k] = r * cos(th);
                nrm[2 * k + 1] = r * sin(th);
            }
            int inside = 1;
            for (int j = 0; j < d; ++j) {
                q[j] = PI * (p->prop_mu[c * 8 + j] + p->prop_sd[c * 8 + j] * nrm[j]);
                if (q[j] < sc->q_lo[j] || q[j] > sc->q_hi[j]) inside = 0;
            }
            ylearn_t = 60.0 * (p->prop_mu[c * 8 + 7] + p->prop_sd[c * 8 + 7] * nrm[7]);
            if (!inside) fl |= ORC_SKIP;
        }
        if (sc->variant == ORC_IR) {
            g = index24(u[0], N);
            if (!(p->L < Ubar)) {
                fl |= ORC_SKIP;
            } else if (use_net) {
                /* T from the arrival histogram over [t_min, t_max]; the group is
                 * the one whose uniform interval holds T */
                int b = 0;
                while (b < 31 && !(unit24(u[15]) < p->prop_hcum[b])) ++b;
                double wb = (sc->t_max - sc->t_min) / 32.0;
                Tw = sc->t_min + ((double)b + unit24(u[24])) * wb;
                if (!(Tw >= p->L && Tw < Ubar)) {
                    fl |= ORC_SKIP;
                } else {
                    int gi = (int)floor((Tw - p->L) / ((Ubar - p->L) / N));
                    g = gi < 0 ? 0 : (gi >= N ? N - 1 : gi);
                    if (!(fl & ORC_SKIP)) {
                        double xg[ORC_MAX_DOF + 1];
                        for (int j = 0; j < d; ++j) xg[j] = sc->q_g[j];
                        xg[d] = Tw;
                        if (!orc_state_valid(sc, xg, NULL)) fl |= ORC_SKIP;
                        double lo = config_dist(d, sc->q_s, q) / v;
                        double hi = Tw - config_dist(d, q, sc->q_g) / v;
                        trw = ylearn_t;
                        if (hi < lo || !(trw >= lo && trw <= hi)) fl |= ORC_SKIP;
                        if (dr == 1 && (!gact[g] || unit24(u[12]) <= sc->p_new)) fl |= ORC_USE_NEW;
                    }
                }
            } else {
                if (unit24(u[1]) < sc->p_guided && p->np[g] > 0) {
                    /* pick a guided portion with probability proportional to its length */
                    double Gi = 0.0;
                    const double *pc = p->pieces + (size_t)g * ORC_MAXP * 2;
                    for (int k = 0; k < p->np[g]; ++k) Gi += pc[2 * k + 1] - pc[2 * k];
                    double c = unit24(u[2]) * Gi, acc = 0.0;
                    int sel = p->np[g] - 1;
                    for (int k = 0; k < p->np[g]; ++k) {
                        acc += pc[2 * k + 1] - pc[2 * k];
                        if (c < acc) { sel = k; break; }
                    }
                    Tw = pc[2 * sel] + unit24(u[3]) * (pc[2 * sel + 1] - pc[2 * sel]);
                } else {
                    Tw = p->I[2 * g] + unit24(u[3]) * (p->I[2 * g + 1] - p->I[2 * g]);
                }
                /* the proposed root (q_g, T) is collision-checked at its time */
                double xg[ORC_MAX_DOF + 1];
                for (int j = 0; j < d; ++j) xg[j] = sc->q_g[j];
                xg[d] = Tw;
                if (!orc_state_valid(sc, xg, NULL)) fl |= ORC_SKIP;
                /* Eq. 6: t_r ~ U[D(q_s,q_r)/v, T - D(q_r,q_g)/v], empty -> reject */
                double lo = config_dist(d, sc->q_s, q) / v;
                double hi = Tw - config_dist(d, q, sc->q_g) / v;
                if (hi < lo) fl |= ORC_SKIP;
                else trw = lo + unit24(u[11]) * (hi - lo);
                if (dr == 1 && (!gact[g] || unit24(u[12]) <= sc->p_new)) fl |= ORC_USE_NEW;
            }
        } else {
            if (dr == 1) {
                int64_t k = w >> 1;
                if (p->n_active == 0) {
                    fl |= ORC_SKIP;
                } else {
                    g = p->active_list[k % p->n_active];
                    Tw = p->slotT[g];
                }
            }
        }
        dir[w] = dr;
        flags[w] = fl;
        grp[w] = g;
        T[w] = Tw;
        for (int j = 0; j < d; ++j) qr[(int64_t)j * B + w] = q[j];
        tr[w] = trw;
    }
}

/* ========================================================================= */
/* One extend batch (Alg. 1 for every worker against the snapshot taken at   */
/* entry; reading: inserts are committed in worker order after all workers   */
/* ran), then the incumbent update and the allocation update.                */
/* ========================================================================= */

typedef struct {
    int8_t status;
    int pool;
    int64_t parent;          /* NN node (global), or -1 for a virtual root */
    double xn[ORC_MAX_DOF + 1];
    double xnew[ORC_MAX_DOF + 1];
    double cost, rootT;
    int64_t bridge;
    uint8_t bridge_ok;
    double Up, Cp;
    uint8_t amb;
    int64_t newid;           /* committed index of x_new, or -1 */
} orc_work;

/* Best-ranked bridge from x (new node, direction sigma) into the opposite
 * set of the snapshot: candidates satisfy the time direction and the speed
 * bound; rank by arrival time, then rho, then index (lowest wins). */
static int64_t best_bridge(const orc_planner *p, const int64_t *cnt, double U, int sigma, const double *x,
                           double x_rootT, double *arr_out, uint8_t *amb) {
    const orc_scene *sc = &p->sc;
    int d = sc->d, w = d + 1;
    int64_t best = -1;
    double ba = INF, br = INF;
    *amb = 0;
    int pool_lo = sigma > 0 ? 1 : 0, pool_hi = sigma > 0 ? p->n_pools : 1;
    /* pass 1: best key */
    for (int pool = pool_lo; pool < pool_hi; ++pool) {
        if (sc->variant == ORC_RR && pool > 0 && !p->slot_active[pool - 1]) continue;
        for (int64_t i = 0; i < cnt[pool]; ++i) {
            int64_t idx = p->base[pool] + i;
            const double *y = p->x + idx * w;
            if (sigma > 0 && sc->variant == ORC_IR && !(p->rootT[idx] < U)) continue;
            double arr = sigma > 0 ? p->rootT[idx] : x_rootT;
            /* the candidate must be reachable from x in direction sigma */
            double r = orc_rho(d, sc->v_max, sigma, x, y);
            if (isinf(r)) continue;
            if (arr < ba || (arr == ba && r < br)) { ba = arr; br = r; best = idx; }
        }
    }
    /* fragility: a different candidate with equal arrival and rho within 1e-5,
     * or one near the speed cone */
    if (best >= 0) {
        for (int pool = pool_lo; pool < pool_hi && !*amb; ++pool) {
            if (sc->variant == ORC_RR && pool > 0 && !p->slot_active[pool - 1]) continue;
            for (int64_t i = 0; i < cnt[pool] && !*amb; ++i) {
                int64_t idx = p->base[pool] + i;
                if (idx == best) continue;
                const double *y = p->x + idx * w;
                if (sigma > 0 && sc->variant == ORC_IR && !(p->rootT[idx] < U)) continue;
                double arr = sigma > 0 ? p->rootT[idx] : x_rootT;
                if (arr != ba) continue;
                double D = config_dist(d, x, y);
                double del = sigma * (y[d] - x[d]);
                double vd = sc->v_max * del;
                double raw = sqrt((D * D + (y[d] - x[d]) * (y[d] - x[d]) * sc->v_max * sc->v_max) / 2.0);
                double r = orc_rho(d, sc->v_max, sigma, x, y);
                double lim = br * (1.0 + 1e-5) + 1e-12;
                if (r <= lim) *amb = 1;
                if (del > 0.0 && fabs(D * D - vd * vd) <= 1e-5 * vd * vd && raw <= lim) *amb = 1;
            }
        }
    }
    *arr_out = ba;
    return best;
}

/* The best-ranked bridge from state x (direction sigma, root time x_rootT of
 * x's own tree) into the opposite set of the planner's current trees, as the
 * extend step selects it (test access to the ranking).  Returns the global
 * index or -1; arr receives the candidate's arrival time. */
int64_t orc_planner_bridge(const orc_planner *p, int sigma, const double *x, double x_rootT, double *arr,
                           uint8_t *amb) {
    return best_bridge(p, p->count, p->U, sigma, x, x_rootT, arr, amb);
}

/* A strict drop of the incumbent arrival to U outside the extend step, for
 * the recycling variant (test access to the Alg. 3 allocation update):
 * U is set and the roots are deactivated and recycled as after an improving
 * iteration.  Returns 0, or -1 for an interval-root planner or U not below
 * the current incumbent. */
int orc_planner_recycle(orc_planner *p, double U) {
    if (p->sc.variant != ORC_RR || !(U < p->U)) return -1;
    p->U = U;
    rr_update(p);
    return 0;
}

int orc_planner_extend(orc_planner *p, int64_t B, const int8_t *dir, const uint8_t *flags, const int32_t *grp,
                       const double *T, const double *qr, const double *tr,
                       /* outputs (any may be NULL) */
                       int8_t *status, int32_t *parent_out, int32_t *new_idx, double *xnew_out /* (d+1) x B */,
                       int32_t *bridge_out, uint8_t *bridge_ok, double *Up_out, double *Cp_out, uint8_t *amb_out,
                       double *edge_margin, double *bridge_margin) {
    const orc_scene *sc = &p->sc;
    int d = sc->d, w = d + 1;
    double v = sc->v_max, H = p->H;
    int64_t cnt[1 + 256];
    memcpy(cnt, p->count, sizeof(int64_t) * (size_t)p->n_pools);
    double U0 = p->U;
    orc_work *wk = (orc_work *)calloc((size_t)B, sizeof(orc_work));
    for (int64_t i = 0; i < B; ++i) {
        orc_work *k = &wk[i];
        k->parent = -1;
        k->newid = -1;
        k->bridge = -1;
        k->Up = INF;
        k->Cp = INF;
        if (edge_margin) edge_margin[i] = INF;
        if (bridge_margin) bridge_margin[i] = INF;
        if (flags[i] & ORC_SKIP) { k->status = ORC_ST_SKIPPED; continue; }
        int sigma = dir[i] == 0 ? 1 : -1;
        double xr[ORC_MAX_DOF + 1];
        for (int j = 0; j < d; ++j) xr[j] = qr[(int64_t)j * B + i];
        xr[d] = tr[i];
        k->pool = dir[i] == 0 ? 0 : 1 + grp[i];
        int virt = 0;
        int64_t nn = -1;
        double rho = INF;
        if (sc->variant == ORC_IR) {
            if (dir[i] == 1 && (flags[i] & ORC_USE_NEW)) {
                virt = 1;
                for (int j = 0; j < d; ++j) k->xn[j] = sc->q_g[j];
                k->xn[d] = T[i];
                rho = orc_rho(d, v, sigma, k->xn, xr);
            } else {
                int pool = k->pool;
                int64_t n = cnt[pool];
                uint8_t *mask = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
                for (int64_t a = 0; a < n; ++a) {
                    int64_t idx = p->base[pool] + a;
                    mask[a] = (uint8_t)(pool == 0 || p->rootT[idx] < U0);
                }
                nn = orc_nearest(sc, n, p->x + p->base[pool] * w, mask, sigma, ORC_METRIC_RHO, xr, &rho, &k->amb);
                free(mask);
                if (nn >= 0) {
                    nn += p->base[pool];
                    memcpy(k->xn, p->x + nn * w, sizeof(double) * (size_t)w);
                }
            }
            if (isinf(rho)) { k->status = ORC_ST_TRAPPED; continue; }
            /* Alg. 1: alpha = min(1, eta / rho), same fraction in q and t */
            double alpha = fmin(1.0, sc->eta / rho);
            for (int c = 0; c <= d; ++c) k->xnew[c] = k->xn[c] + alpha * (xr[c] - k->xn[c]);
        } else {
            int pool = k->pool;
            int64_t n = cnt[pool];
            double Dn = INF;
            if (n > 0) {
                nn = orc_nearest(sc, n, p->x + p->base[pool] * w, NULL, sigma, ORC_METRIC_CONFIG, xr, &Dn, &k->amb);
                if (nn >= 0) nn += p->base[pool];
            }
            /* "no proposal": empty tree or a zero-length step */
            if (nn < 0 || !(Dn > 0.0)) { k->status = ORC_ST_TRAPPED; continue; }
            memcpy(k->xn, p->x + nn * w, sizeof(double) * (size_t)w);
            /* Eq. 8: configuration step capped at eta, timed at maximum speed */
            double f = fmin(1.0, sc->eta / Dn);
            for (int j = 0; j < d; ++j) k->xnew[j] = k->xn[j] + f * (xr[j] - k->xn[j]);
            k->xnew[d] = k->xn[d] + sigma * config_dist(d, k->xn, k->xnew) / v;
        }
        if (!(k->xnew[d] >= 0.0 && k->xnew[d] <= H)) { k->status = ORC_ST_TRAPPED; continue; }
        int32_t fh;
        double em;
        int ok = orc_edge_check(sc, k->xn, k->xnew, &fh, NULL, &em, NULL);
        p->n_edge_checks++;
        if (edge_margin) edge_margin[i] = em;
        if (!ok) { k->status = ORC_ST_TRAPPED; continue; }
        k->status = ORC_ST_ADVANCED;
        k->parent = nn;
        double step = config_dist(d, k->xn, k->xnew);
        if (dir[i] == 0) {
            k->cost = p->cost[nn] + step;
            k->rootT = 0.0;
        } else if (virt) {
            k->cost = step;
            k->rootT = T[i];
        } else {
            k->cost = p->cost[nn] + step;
            k->rootT = p->rootT[nn];
        }
        /* best-ranked bridge into the opposite set, then its collision check */
        double arr;
        uint8_t bamb;
        int64_t b = best_bridge(p, cnt, U0, sigma, k->xnew, k->rootT, &arr, &bamb);
        k->amb |= bamb;
        k->bridge = b;
        if (b >= 0) {
            double bm;
            int bok = orc_edge_check(sc, k->xnew, p->x + b * w, NULL, NULL, &bm, NULL);
            p->n_bridge_checks++;
            if (bridge_margin) bridge_margin[i] = bm;
            k->bridge_ok = (uint8_t)bok;
            if (bok) {
                double link = config_dist(d, k->xnew, p->x + b * w);
                k->Up = arr;
                k->Cp = k->cost + link + p->cost[b];
            }
        }
    }
    /* commit in worker order.  Reading of capacity (the paper does not
     * bound the trees): the workers of a pool claim consecutive slots in
     * worker order, a dropped worker's claim included, as an atomic slot
     * counter would hand them out; a worker whose claim ends past the pool's
     * capacity is dropped, so once one worker is dropped every later worker
     * of that pool is dropped too (a suffix in worker order). */
    int64_t claimed[1 + 256];
    memcpy(claimed, p->count, sizeof(int64_t) * (size_t)p->n_pools);
    int64_t best_w = -1;
    for (int64_t i = 0; i < B; ++i) {
        orc_work *k = &wk[i];
        int32_t nid = -1;
        if (k->status == ORC_ST_ADVANCED) {
            int pool = k->pool;
            int need = k->parent < 0 ? 2 : 1;
            claimed[pool] += need;
            if (claimed[pool] > p->cap[pool]) {
                k->status = ORC_ST_DROPPED;
                p->overflow = 1;
            } else {
                int64_t par = k->parent;
                if (par < 0) par = push_node(p, pool, k->xn, -1, 0.0, k->rootT); /* materialize the tree */
                k->parent = par;
                nid = (int32_t)push_node(p, pool, k->xnew, (int32_t)par, k->cost, k->rootT);
                if (k->bridge_ok && (best_w < 0 || k->Up < wk[best_w].Up ||
                                     (k->Up == wk[best_w].Up && k->Cp < wk[best_w].Cp)))
                    best_w = i;
            }
        }
        if (status) status[i] = k->status;
        if (parent_out) parent_out[i] = (int32_t)k->parent;
        if (new_idx) new_idx[i] = nid;
        if (xnew_out)
            for (int c = 0; c <= d; ++c) xnew_out[(int64_t)c * B + i] = k->status >= ORC_ST_ADVANCED ? k->xnew[c] : 0.0;
        if (bridge_out) bridge_out[i] = (int32_t)k->bridge;
        if (bridge_ok) bridge_ok[i] = k->bridge_ok;
        if (Up_out) Up_out[i] = k->Up;
        if (Cp_out) Cp_out[i] = k->Cp;
        if (amb_out) amb_out[i] = k->amb;
        k->newid = nid;
    }
    int improved = 0;
    if (best_w >= 0) {
        orc_work *k = &wk[best_w];
        if (k->Up < p->U || (k->Up == p->U && k->Cp < p->C)) {
            int strict = k->Up < p->U;
            p->U = k->Up;
            p->C = k->Cp;
            if (dir[best_w] == 0) { p->inc_f = k->newid; p->inc_b = k->bridge; }
            else { p->inc_f = k->bridge; p->inc_b = k->newid; }
            if (p->first_iter < 0) p->first_iter = p->iter;
            improved = strict ? 2 : 1;
        }
    }
    if (improved == 2) {
        if (sc->variant == ORC_IR) ir_repartition(p);
        else rr_update(p);
    }
    p->iter++;
    free(wk);
    return improved;
}

/* ========================================================================= */
/* Planner loop (Alg. 2 / Alg. 3) and path extraction.                       */
/* ========================================================================= */

static int is_trivial(const orc_planner *p) {
    const orc_scene *sc = &p->sc;
    for (int j = 0; j < sc->d; ++j)
        if (sc->q_s[j] != sc->q_g[j]) return 0;
    double xs[ORC_MAX_DOF + 1];
    for (int j = 0; j < sc->d; ++j) xs[j] = sc->q_s[j];
    xs[sc->d] = 0.0;
    /* reading: the trivial return applies when arrival at time 0 is allowed */
    return p->L <= 0.0 && orc_state_valid(sc, xs, NULL);
}

/* Runs up to max_iters iterations (Alg. 2 stops early once L >= min(H, U)).
 * Returns 0 when a path was found, 1 when none, 2 for the trivial case. */
int orc_planner_run(orc_planner *p, int64_t max_iters) {
    const orc_scene *sc = &p->sc;
    if (is_trivial(p)) { p->U = 0.0; p->C = 0.0; return 2; }
    double xs[ORC_MAX_DOF + 1];
    for (int j = 0; j < sc->d; ++j) xs[j] = sc->q_s[j];
    xs[sc->d] = 0.0;
    if (!orc_state_valid(sc, xs, NULL)) return 1;
    int64_t B = sc->batch;
    int d = sc->d;
    int8_t *dir = (int8_t *)malloc((size_t)B);
    uint8_t *fl = (uint8_t *)malloc((size_t)B);
    int32_t *g = (int32_t *)malloc(sizeof(int32_t) * (size_t)B);
    double *T = (double *)malloc(sizeof(double) * (size_t)B);
    double *qr = (double *)malloc(sizeof(double) * (size_t)B * d);
    double *tr = (double *)malloc(sizeof(double) * (size_t)B);
    for (int64_t it = 0; it < max_iters; ++it) {
        if (sc->variant == ORC_IR && !(p->L < fmin(p->H, p->U))) break;
        orc_planner_sample(p, p->iter, B, dir, fl, g, T, qr, tr);
        orc_planner_extend(p, B, dir, fl, g, T, qr, tr, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL,
                           NULL);
    }
    free(dir); free(fl); free(g); free(T); free(qr); free(tr);
    return isinf(p->U) ? 1 : 0;
}

/* Path = forward chain root..v_f, then the backward chain w_b..root.
 * states: caller buffer of max_n x (d+1).  Returns the number of states or -1. */
int64_t orc_planner_path(const orc_planner *p, int64_t max_n, double *states) {
    int w = p->sc.d + 1;
    if (p->inc_f < 0 || p->inc_b < 0) return -1;
    int64_t nf = 0;
    for (int64_t i = p->inc_f; i >= 0; i = p->parent[i]) ++nf;
    if (nf > max_n) return -1;
    /* forward chain written back to front so that it runs root -> v_f */
    int64_t j = nf - 1;
    for (int64_t i = p->inc_f; i >= 0; i = p->parent[i], --j)
        memcpy(states + j * w, p->x + i * w, sizeof(double) * (size_t)w);
    int64_t n = nf;
    for (int64_t i = p->inc_b; i >= 0; i = p->parent[i]) {
        if (n >= max_n) return -1;
        memcpy(states + n * w, p->x + i * w, sizeof(double) * (size_t)w);
        ++n;
    }
    return n;
}

/* ------------------------------------------------------------------------- */
/* Accessors and snapshot import/export (test I/O).                          */
/* ------------------------------------------------------------------------- */

void orc_planner_info(const orc_planner *p, double *out /* 16 */) {
    out[0] = p->U;
    out[1] = p->C;
    out[2] = (double)p->inc_f;
    out[3] = (double)p->inc_b;
    out[4] = (double)p->first_iter;
    out[5] = p->L;
    out[6] = p->H;
    out[7] = (double)p->k_lo;
    out[8] = (double)p->k_hi;
    out[9] = (double)p->iter;
    out[10] = (double)p->overflow;
    out[11] = (double)p->n_active;
    out[12] = (double)p->total;
    out[13] = (double)p->n_pools;
    out[14] = (double)p->n_edge_checks;
    out[15] = (double)p->n_bridge_checks;
}

void orc_planner_counts(const orc_planner *p, int64_t *counts) {
    memcpy(counts, p->count, sizeof(int64_t) * (size_t)p->n_pools);
}

void orc_planner_goal_free(const orc_planner *p, uint8_t *out) {
    memcpy(out, p->gfree, (size_t)(p->k_hi - p->k_lo + 1));
}

void orc_planner_partition(const orc_planner *p, double *I, int32_t *np, double *pieces, int maxp) {
    int N = p->sc.n_groups;
    memcpy(I, p->I, sizeof(double) * 2 * (size_t)N);
    memcpy(np, p->np, sizeof(int32_t) * (size_t)N);
    for (int g = 0; g < N; ++g)
        for (int k = 0; k < p->np[g] && k < maxp; ++k) {
            pieces[((size_t)g * maxp + k) * 2] = p->pieces[((size_t)g * ORC_MAXP + k) * 2];
            pieces[((size_t)g * maxp + k) * 2 + 1] = p->pieces[((size_t)g * ORC_MAXP + k) * 2 + 1];
        }
}

void orc_planner_slots(const orc_planner *p, double *T, int32_t *active, uint32_t *gen, int64_t *kidx) {
    int N = p->sc.n_groups;
    for (int s = 0; s < N; ++s) {
        T[s] = p->slotT[s];
        active[s] = p->slot_active[s];
        gen[s] = p->slot_gen[s];
        kidx[s] = p->slotK[s];
    }
}

/* Export the node arrays of pool range: x (n x (d+1)), parent, cost, rootT. */
void orc_planner_export(const orc_planner *p, double *x, int32_t *parent, double *cost, double *rootT) {
    int w = p->sc.d + 1;
    memcpy(x, p->x, sizeof(double) * (size_t)(p->total * w));
    memcpy(parent, p->parent, sizeof(int32_t) * (size_t)p->total);
    memcpy(cost, p->cost, sizeof(double) * (size_t)p->total);
    memcpy(rootT, p->rootT, sizeof(double) * (size_t)p->total);
}

/* Replace the planner state by a snapshot (counts per pool; node arrays in
 * global numbering; incumbent; recycling slots).  slot arrays may be NULL for
 * interval root.  The allocation (partition / active list) is recomputed. */
void orc_planner_import(orc_planner *p, const int64_t *counts, const double *x, const int32_t *parent,
                        const double *cost, const double *rootT, double U, double C, int64_t inc_f, int64_t inc_b,
                        int64_t iter, const double *slotT, const int32_t *slot_active, const uint32_t *slot_gen,
                        const int64_t *slotK) {
    int w = p->sc.d + 1;
    memcpy(p->count, counts, sizeof(int64_t) * (size_t)p->n_pools);
    memcpy(p->x, x, sizeof(double) * (size_t)(p->total * w));
    memcpy(p->parent, parent, sizeof(int32_t) * (size_t)p->total);
    memcpy(p->cost, cost, sizeof(double) * (size_t)p->total);
    memcpy(p->rootT, rootT, sizeof(double) * (size_t)p->total);
    p->U = U;
    p->C = C;
    p->inc_f = inc_f;
    p->inc_b = inc_b;
    p->iter = iter;
    if (p->sc.variant == ORC_IR) {
        ir_repartition(p);
    } else {
        for (int s = 0; s < p->sc.n_groups; ++s) {
            p->slotT[s] = slotT[s];
            p->slot_active[s] = slot_active[s];
            p->slot_gen[s] = slot_gen[s];
            p->slotK[s] = slotK[s];
        }
        rr_refresh_active(p);
    }
}

/* ========================================================================= */
/* Path validator: every returned path is re-checked here.                   */
/* ========================================================================= */

int orc_validate_path(const orc_scene *sc, int64_t n, const double *st, double U, double C, double rel_tol,
                      char *msg, int msglen) {
    int d = sc->d, w = d + 1;
    double L = orc_lower_bound(sc);
#define FAIL(...) do { if (msg) snprintf(msg, (size_t)msglen, __VA_ARGS__); return 0; } while (0)
    if (n < 1) FAIL("empty path");
    for (int j = 0; j < d; ++j)
        if (fabs(st[j] - sc->q_s[j]) > 1e-6) FAIL("first state is not q_s (dim %d)", j);
    if (fabs(st[d]) > 1e-9) FAIL("first state time %g != 0", st[d]);
    const double *last = st + (n - 1) * w;
    for (int j = 0; j < d; ++j)
        if (fabs(last[j] - sc->q_g[j]) > 1e-6) FAIL("last state is not q_g (dim %d)", j);
    if (fabs(last[d] - U) > 1e-6 * fmax(1.0, U)) FAIL("last time %.9g != U %.9g", last[d], U);
    if (n > 1 && (U < L - 1e-6 * fmax(1.0, L) || U > sc->t_max + 1e-6)) FAIL("U %.9g outside [%.9g, %.9g]", U, L, sc->t_max);
    double len = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        const double *a = st + i * w, *b = st + (i + 1) * w;
        double dtt = b[d] - a[d];
        if (!(dtt > 0.0)) FAIL("time not increasing at segment %lld (%.9g -> %.9g)", (long long)i, a[d], b[d]);
        double D = config_dist(d, a, b);
        if (D > sc->v_max * dtt * (1.0 + rel_tol) + 1e-9) FAIL("speed bound violated at segment %lld: D=%.9g v*dt=%.9g", (long long)i, D, sc->v_max * dtt);
        int32_t fh;
        if (!orc_edge_check(sc, a, b, &fh, NULL, NULL, NULL)) FAIL("segment %lld collides at state %d", (long long)i, fh);
        len += D;
    }
    double x0[ORC_MAX_DOF + 1];
    memcpy(x0, st, sizeof(double) * (size_t)w);
    if (!orc_state_valid(sc, x0, NULL)) FAIL("start state invalid");
    if (fabs(len - C) > rel_tol * fmax(1.0, len) + 1e-6) FAIL("length %.9g != C %.9g", len, C);
#undef FAIL
    if (msg && msglen > 0) msg[0] = 0;
    return 1;
}
