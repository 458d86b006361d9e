/*
 * pf_dem.h -- C ABI of the many-sphere rigid-body run whose pairwise capillary-bridge forces come
 * from the learned surrogate (pf_mlp.h) instead of a field solve.
 *
 * N spheres in a periodic cube move under pairwise bridge forces and a linear spring-dashpot
 * contact force, integrated with the semi-implicit Euler update of the rigid bodies (Sec. 3.3:
 * velocity from the force first, then position from the new velocity).  Sec. 2.2 fixes a bridge
 * between two spheres by the surface gap, the two radii, the liquid volume and the contact angle;
 * here a bridge joins every pair whose surface gap is below gap_max, and its force is attractive
 * along the line of centres with magnitude
 *
 *     F = f * R*,   f = y * out_scale + out_shift,   R* = 2 R_i R_j / (R_i + R_j),
 *
 * y the network's output for the input row (feature_k - in_shift[k]) * in_scale[k] of the
 * features (max(gap, gap_min) / R*, min(R_i, R_j) / max(R_i, R_j), V_L / R*^3, theta) with
 * V_L = c / (1 - c) * (4/3) pi (R_i^3 + R_j^3), c the liquid fraction of Sec. 2.2.  Bridge and
 * contact forces act along the line of centres, so no torque arises and only translations are
 * integrated.  Per-sphere force sums run in a fixed order in FP64 (results do not depend on
 * scheduling); the network runs in BF16 with FP32 accumulation.
 *
 * A pair force can be overridden from the host (pf_dem_set_overrides): the run then uses the
 * given value for that pair instead of the network's, e.g. the force of a field re-solve of the
 * pair when the network's error on it is too large.
 *
 * Conventions as in pf_lbm.h: status returns, caller-owned 256-byte-aligned device workspace
 * (workspace == NULL queries its size), one stream per handle, no thread safety.  The network
 * handle must be bound to the same stream, and must stay alive while the run uses it; its
 * max_batch must be at least max_pairs.
 */
#ifndef PF_DEM_H
#define PF_DEM_H

#include <stddef.h>
#include <stdint.h>

#include "pf_lbm.h"
#include "pf_mlp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pf_dem pf_dem;

typedef struct {
    uint32_t struct_size;   /* sizeof(pf_dem_config)                                          */
    int32_t n;              /* spheres, 2..16384                                              */
    int32_t max_neighbours; /* bridged partners per sphere, 1..64                             */
    int32_t max_pairs;      /* bridged pairs, 1..65536                                        */
    double box;             /* edge of the periodic cube, > 2 max radius + gap_max            */
    double dt;              /* time step, > 0                                                 */
    double density;         /* sphere mass density: m = density (4/3) pi R^3, > 0             */
    double k_n;             /* contact spring: force k_n * overlap, >= 0                      */
    double gamma_n;         /* contact dashpot: force gamma_n * approach speed, >= 0          */
    double theta;           /* contact angle of every bridge (radians), 0..pi/2               */
    double liquid_fraction; /* c of every bridge, 0 < c < 1                                   */
    double gap_min;         /* surface gaps below this are evaluated at gap_min, >= 0         */
    double gap_max;         /* pairs with surface gap >= gap_max carry no bridge, > gap_min   */
    float in_shift[4], in_scale[4]; /* network input normalisation                            */
    float out_shift, out_scale;     /* network output de-normalisation                        */
} pf_dem_config;

/* Create a run.  radii [n], x0 [n][3] (in [0, box)), v0 [n][3] are HOST arrays; net a network
 * with n_in == 4 bound to hip_stream.  Errors: EINVAL (bad configuration or arguments), ENOMEM
 * (workspace too small, host allocation), EDEVICE. */
int pf_dem_init(const pf_dem_config *cfg, const double *radii, const double *x0, const double *v0, pf_mlp *net,
                void *workspace, size_t ws_bytes, void *hip_stream, pf_dem **out, size_t *ws_bytes_needed);

/* Bridge list, network forces and per-sphere force sums at the current positions, no motion.
 * Synchronises once (to size the network's batch).  ENOMEM when a sphere has more than
 * max_neighbours partners or the run more than max_pairs bridges (the state is unchanged). */
int pf_dem_evaluate(pf_dem *h);

/* n_steps x (pf_dem_evaluate, then v += F / m dt, x += v dt, wrapped into the box). */
int pf_dem_step(pf_dem *h, int32_t n_steps);

/* Current state, HOST arrays of [n][3] (any may be NULL): positions, velocities and the forces of
 * the last evaluation.  Synchronises. */
int pf_dem_state(pf_dem *h, double *x, double *v, double *f);

/* Bridges of the last evaluation, ordered by (i, j), i < j: ij [k][2], features [k][4] (the
 * unnormalised network features above), force [k] (the force F used, override included).
 * HOST arrays of max_out rows; *n_out receives the number of bridges (rows beyond max_out are not
 * written).  Synchronises. */
int pf_dem_pairs(pf_dem *h, int32_t max_out, int32_t *ij, double *features, double *force, int32_t *n_out);

/* Replace the overrides: n pairs (i, j) (either order) with force[k] used instead of the network
 * while the pair stays bridged; n == 0 clears them.  n <= 256.  Synchronises. */
int pf_dem_set_overrides(pf_dem *h, int32_t n, const int32_t *ij, const double *force);

void pf_dem_destroy(pf_dem *h);
const char *pf_dem_last_error(const pf_dem *h);

#ifdef __cplusplus
}
#endif

#endif /* PF_DEM_H */
