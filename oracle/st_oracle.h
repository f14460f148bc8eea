/*
 * st_oracle.h -- FP64 CPU oracle for the ST-pRRTC space-time extend path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference the
 * HIP path is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product library never links,
 * includes or calls anything here, and this code includes nothing from the
 * product.  Everything is scalar double precision, single-threaded, and
 * follows the paper's definitions in the order the paper states them:
 *
 *   Sec. III (Eq. 1-4)   state space, minimum travel time, feasibility
 *   Sec. IV-A            shared forward tree + backward forest, incumbent (U,C)
 *   Sec. IV-B (Eq. 5-7)  goal-time bound, guided windows, N groups, conditional
 *                        query time, directed space-time distance, Alg. 1 / 2
 *   Sec. V   (Eq. 8)     root recycling, maximum-speed extension, Alg. 3
 *   Sec. VI              obstacles interpolated at absolute query times;
 *                        the arm's own links and fixed boxes (pRRTC's sphere
 *                        checker lineage) as time-independent terms
 *
 * Readings of passages the paper leaves open are listed at each function.
 */
#ifndef ST_ORACLE_H
#define ST_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_DOF 7
#define ORC_MAX_SPH 128
#define ORC_MAX_OBS 64
#define ORC_MAX_WP 32
#define ORC_MAX_SELF 32
#define ORC_MAX_BOX 16

enum { ORC_KIND_TRANSLATE = 0, ORC_KIND_DH = 1 };
enum { ORC_IR = 0, ORC_RR = 1 };
enum { ORC_METRIC_RHO = 0, ORC_METRIC_CONFIG = 1 };

/* sample flags */
enum { ORC_SKIP = 1, ORC_USE_NEW = 2, ORC_LEARNED = 4 };
/* extend status */
enum { ORC_ST_SKIPPED = 0, ORC_ST_TRAPPED = 1, ORC_ST_ADVANCED = 2, ORC_ST_DROPPED = 3 };

typedef struct orc_scene {
    int32_t d, kind;
    double dh[ORC_MAX_DOF][4];          /* a, alpha, d, theta0 (standard DH) */
    int32_t n_sph;
    int32_t sph_link[ORC_MAX_SPH];      /* 0 = base frame, l = frame after joint l */
    double sph[ORC_MAX_SPH][4];         /* local x, y, z, radius */
    double q_lo[ORC_MAX_DOF], q_hi[ORC_MAX_DOF];
    double q_s[ORC_MAX_DOF], q_g[ORC_MAX_DOF];
    double t_min, t_max, v_max;         /* arrival range [t_min, t_max], H = t_max */
    int32_t n_obs;
    int32_t n_wp[ORC_MAX_OBS];
    double wp[ORC_MAX_OBS][ORC_MAX_WP][4]; /* t, x, y, z */
    double obs_r[ORC_MAX_OBS];
    /* planner parameters */
    int32_t variant, n_groups, batch;
    double eta, h, dt, p_new, p_guided;
    int32_t cap_fwd, cap_bwd;
    uint32_t seed, problem_id;
    int32_t no_recycling;               /* recycling variant: 1 = roots fixed, deactivation only (ablation) */
    /* static geometry (arms): link pairs tested against each other, and
     * fixed oriented boxes.  A pair (la, lb) tests every sphere of link la
     * against every sphere of link lb.  A box row is centre (3), half
     * extents (3), then its three unit axes in world coordinates (3 x 3,
     * one axis per row). */
    int32_t n_self;
    int32_t self_pair[ORC_MAX_SELF][2];
    int32_t n_box;
    double box[ORC_MAX_BOX][15];
} orc_scene;

typedef struct orc_planner orc_planner;

#ifdef __cplusplus
}
#endif
#endif
