/*
 * pf_lbm.h -- C interface of the MI355X coupled multi-phase-field / lattice-Boltzmann step.
 *
 * Method: R. Schiedung, M. Tegeler, D. Medvedev, F. Varnik, "Simulation of Capillary-Driven
 * Kinetics with Multi-Phase-Field and Lattice-Boltzmann Method" (arXiv:1902.10432), Sec. 3.
 *
 * One handle holds one periodic box (lattice spacing and time step 1) with nb rigid bodies, each
 * represented by one solid phase field phi_a (a = 0..nb-1); the fluid phase fraction is
 * 1 - sum_a phi_a (Sec. 3.1).  One call of the step advances, in this order:
 *   pseudopotential force with solid wetting (Sec. 3.2.3), Guo-forced BGK collision (Sec. 3.2.1),
 *   streaming with half-way bounce-back from moving walls, rest-population mass correction and
 *   momentum exchange (Sec. 3.2.2), solid-solid repulsion (Sec. 3.1.2), rigid-body update
 *   (Sec. 3.1.1), split MC-limited advection of each phase field with its body's rigid velocity
 *   (Sec. 3.1.1, 3.3), multi-phase-field kinetics with the volume-restoring driving force
 *   (Sec. 3.3), solid/fluid reclassification and node conversion (Sec. 3.2.2).
 *
 * Conventions
 *   - Every function returns a status (PF_LBM_OK or a negative code) and never throws; the
 *     message of the last failure is available from pf_lbm_last_error (per handle; with a NULL
 *     handle, the message of the last failed pf_lbm_init in this process).
 *   - Memory: the caller owns all device memory.  pf_lbm_init carves one caller-allocated
 *     device workspace; the library calls no device allocator.  Host arrays passed in are read
 *     during the call only.
 *   - Streams: a handle is bound to the HIP stream given at init; pf_lbm_step and pf_lbm_fields
 *     are asynchronous and stream-ordered; pf_lbm_forces synchronises the stream.  A handle is
 *     not thread-safe.
 *   - Fields are x-fastest arrays [nz][ny][nx] (phase fields [nb][nz][ny][nx]).
 */
#ifndef PF_LBM_H
#define PF_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PF_LBM_MAX_BODIES 16

typedef struct pf_lbm pf_lbm; /* opaque handle */

enum {
    PF_LBM_OK = 0,
    PF_LBM_EINVAL = -1,       /* invalid argument or configuration                          */
    PF_LBM_ENOMEM = -2,       /* workspace smaller than required, or a host allocation failed */
    PF_LBM_EUNSUPPORTED = -3, /* valid for the method, not supported by this library        */
    PF_LBM_EDEVICE = -4,      /* a HIP runtime call failed                                  */
    PF_LBM_ENONFINITE = -5,   /* non-finite body force or state, or advection CFL above 1   */
};

/* Velocity sets: D3Q19 (the named workloads) and D3Q27, the set printed in Sec. 3.2.1 (weights
 * 8/27, 2/27, 1/54, 1/216 by speed shell).  Both have c_s^2 = 1/3. */
enum { PF_LBM_D3Q19 = 19, PF_LBM_D3Q27 = 27 };

/* Arithmetic and storage of the fluid populations.  FP64 and FP32 store and compute in that
 * type.  FP16_STORE stores each population f_i(x) as an FP16 deviation from its equilibrium
 * weight at rest, f_i - w_i rho~(x), with rho~(x) = -rho0 log(1 - psi(x)) from the node's
 * pseudopotential of the previous step (its density, up to FP32 rounding), and computes in FP32.
 * In every form the phase fields are FP64, and the per-body force and torque sums, the mass
 * checks and the rigid-body update are FP64. */
enum { PF_LBM_FP64 = 0, PF_LBM_FP32 = 1, PF_LBM_FP16_STORE = 2 };

/* step options (config.flags) */
enum {
    PF_LBM_KINETICS = 1,  /* multi-phase-field kinetics and volume term (Sec. 3.3)        */
    PF_LBM_MOTION = 2,    /* integrate the rigid bodies (Sec. 3.1.1); off = all held still */
    PF_LBM_REPULSION = 4, /* solid-solid repulsion (Sec. 3.1.2)                            */
};

/* pf_lbm_fields selectors */
enum {
    PF_LBM_FIELD_RHO = 0,   /* density sum_i f_i of the post-stream populations; 0 on solid nodes */
    PF_LBM_FIELD_JX = 1,    /* momentum density sum_i c_i f_i (x, y, z); 0 on solid nodes         */
    PF_LBM_FIELD_JY = 2,
    PF_LBM_FIELD_JZ = 3,
    PF_LBM_FIELD_SOLID = 4, /* 1 on solid nodes, 0 on fluid nodes                                 */
    PF_LBM_FIELD_OWNER = 5, /* owning body of a solid node, -1 on fluid nodes                     */
    PF_LBM_FIELD_PSI = 6,   /* pseudopotential of the last step (fluid: psi(rho); solid: psi(varrho)) */
    PF_LBM_FIELD_PHI = 16,  /* PF_LBM_FIELD_PHI + a: phase field of body a                         */
};

/* destination element types of pf_lbm_fields */
enum { PF_LBM_DST_F64 = 0, PF_LBM_DST_F32 = 1 };

typedef struct {
    uint32_t struct_size;   /* sizeof(pf_lbm_config): ABI check                                  */
    int32_t nx, ny, nz;     /* periodic box, cells per axis (each >= 1)                          */
    int32_t lattice;        /* PF_LBM_D3Q19 or PF_LBM_D3Q27                                       */
    int32_t precision;      /* PF_LBM_FP64, PF_LBM_FP32 or PF_LBM_FP16_STORE                      */
    int32_t flags;          /* PF_LBM_KINETICS | PF_LBM_MOTION | PF_LBM_REPULSION                 */
    double tau;             /* BGK relaxation time, > 1/2 (Sec. 3.2.1)                            */
    double G;               /* pseudopotential coupling (Sec. 3.2.3)                              */
    double rho0;            /* reference density of psi = 1 - exp(-rho/rho0), > 0 (Sec. 3.2.3)    */
    double solid_threshold; /* a node is solid iff its fluid fraction is below this (Sec. 3.2.2)  */
    double mobility;        /* M_ab, uniform over pairs (Sec. 3.3)                                */
    double eta;             /* interface width of the kinetics, > 0 (Sec. 3.3)                    */
    const double *sigma;    /* (nb+1) x (nb+1) row-major interface energies, index 0 = fluid      */
                            /* phase; NULL = 1.0 solid/fluid, 0.5 solid/solid (Sec. 3.3)          */
    double r_c, n_exp, e0;  /* repulsion range (0 < r_c <= 4), exponent, strength (Sec. 3.1.2)    */
    double R_A;             /* redistribution radius of node conversion, 1 <= R_A <= sqrt(3)     */
                            /* (Sec. 3.2.2)                                                        */
    double fext[3];         /* uniform external force density on the fluid (0 in the paper)       */
    double phi_floor;       /* resolution of "phi > 0" in the present-phase and interface sets of */
                            /* the kinetics and the volume term (Sec. 3.3), in [0, 0.5): values   */
                            /* at or below it count as absent and the kinetics flushes them to 0; */
                            /* 2^-53 (FP64 unit round-off) is the value used by the workloads,    */
                            /* 0 the literal set                                                  */
} pf_lbm_config;

typedef struct {
    double mass_density; /* rho_a: body mass = rho_a * sum(phi_a) at t = 0 (Sec. 3.3 table)    */
    double wetting_rho;  /* varrho_a: a solid node acts as fluid of this density (Sec. 3.2.3) */
    double v[3];         /* initial translational velocity                                      */
    double w[3];         /* initial angular velocity                                            */
    int32_t fixed;       /* nonzero: the body is never integrated (V, omega, X stay as given)   */
} pf_lbm_body;

/*
 * Create a simulation.
 *   cfg, n_bodies (0..PF_LBM_MAX_BODIES), bodies[n_bodies]: parameters and bodies.
 *   rho0:  HOST FP64 [nz][ny][nx] initial density; the fluid starts at rest, f = f_eq(rho0, 0)
 *          on fluid nodes (values on solid nodes are ignored).
 *   phi0:  HOST FP64 [n_bodies][nz][ny][nx] initial phase fields in [0, 1] with sum <= 1 (may
 *          be NULL when n_bodies == 0).  Body mass, centre (phi-weighted centroid, unwrapped
 *          across the periodic boundary at the largest empty gap of the support), inertia
 *          tensor and reference volume come from phi0.
 *   workspace, ws_bytes: caller-owned device memory, 256-byte aligned.  With workspace == NULL
 *          the call only writes the required size to *ws_bytes_needed and returns PF_LBM_OK.
 *   hip_stream: hipStream_t the handle is bound to (NULL = default stream).
 *   out: receives the handle (owned by the caller, released with pf_lbm_destroy).
 * Errors: PF_LBM_EINVAL (bad sizes or parameters), PF_LBM_ENOMEM (ws_bytes too small),
 *   PF_LBM_EUNSUPPORTED (lattice other than D3Q19/D3Q27, precision other than FP64/FP32/FP16_STORE),
 *   PF_LBM_EDEVICE (HIP failure).  The call returns after the initial fields are on the device.
 */
int pf_lbm_init(const pf_lbm_config *cfg, int32_t n_bodies, const pf_lbm_body *bodies, const double *rho0,
                const double *phi0, void *workspace, size_t ws_bytes, void *hip_stream, pf_lbm **out,
                size_t *ws_bytes_needed);

/* Enqueue n_steps >= 0 time steps on the handle's stream (no host synchronisation).  Returns a
 * pending error from the device (PF_LBM_ENONFINITE) only at the next pf_lbm_forces call. */
int pf_lbm_step(pf_lbm *h, int32_t n_steps);

/*
 * For callers that cannot allocate device memory around a step (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same n_steps >= 0 time steps as
 * pf_lbm_step, bit for bit, with the per-block FP64 force and torque partials of each step taken
 * from a static array the library holds on every GPU it runs on (192 KiB: at most 256 blocks x
 * PF_LBM_MAX_BODIES bodies x 6 values), instead of the handle's workspace.  Kernels are launched
 * one by one on the handle's stream (no HIP graph); the call allocates nothing.  Every call on a
 * GPU shares that GPU's array and every step rewrites the partials it reads, so calls that run one
 * after the other are independent, while calls that overlap in time on one GPU (handles on
 * different streams) race.  Errors: PF_LBM_EINVAL (NULL handle, n_steps < 0, timing enabled),
 * PF_LBM_EUNSUPPORTED (partials beyond the static size), PF_LBM_EDEVICE.
 */
int pf_lbm_step_noalloc(pf_lbm *h, int32_t n_steps);

/*
 * Synchronise the stream and copy the body state to HOST arrays of n_bodies x 3 doubles each
 * (any pointer may be NULL): F, T = total force and torque of the last step (momentum exchange
 * + pseudopotential reaction + repulsion, torques about the centres); X = centre of mass;
 * V = velocity; W = angular velocity (after the last step's update).  Returns
 * PF_LBM_ENONFINITE if the device flagged a non-finite body state or an advection velocity
 * above one cell per step since init.
 */
int pf_lbm_forces(pf_lbm *h, double *F, double *T, double *X, double *V, double *W);

/* Write field `which` (PF_LBM_FIELD_*) of the current state into caller-owned DEVICE memory dst
 * of nz*ny*nx elements of type dst_dtype (PF_LBM_DST_F64 or PF_LBM_DST_F32).  Asynchronous. */
int pf_lbm_fields(pf_lbm *h, int32_t which, void *dst, int32_t dst_dtype);

/* Diagnostics copied to a HOST array of 4 doubles (synchronises): steps taken, fluid-to-solid
 * and solid-to-fluid conversions since init, conversions whose neighbourhood held no fluid node
 * (their mass could not be handed on). */
int pf_lbm_diagnostics(pf_lbm *h, double *out4);

/* Measurement: pf_lbm_timing(h, 1, NULL) starts recording HIP events on the handle's stream
 * around the fused collide-stream kernel and around each whole step of the following
 * pf_lbm_step calls (at most 4096 steps); pf_lbm_timing(h, 0, out4) synchronises, stops and
 * writes to a HOST array of 4 doubles: timed steps, mean collide-stream kernel time (ms), mean
 * step time (ms), and 0 (reserved). */
int pf_lbm_timing(pf_lbm *h, int32_t enable, double *out4);

/* Per-body force and torque history of the last min(steps taken, max_steps, 8192) steps, oldest
 * first, into a HOST array out[n][n_bodies][6] (F x, y, z, then T x, y, z, FP64; the values
 * pf_lbm_forces reports after each of those steps); *n_out receives n.  The device keeps a ring
 * of 8192 steps written inside the step, so a long run needs no host synchronisation per step
 * (the batched sweeps record force histories this way).  Synchronises the handle's stream. */
int pf_lbm_force_history(pf_lbm *h, int32_t max_steps, double *out, int32_t *n_out);

/* Batched stepping of independent simulations (grids of any size): advances each of the n
 * handles by n_steps, launching step pairs round robin over the handles.  Each handle launches
 * on its own stream (given at pf_lbm_init), so the kernels of different instances overlap on the
 * GPU; per instance the result is bit for bit that of pf_lbm_step.  Handles must be distinct.
 * Returns the first error (its message on that handle). */
int pf_lbm_step_batch(pf_lbm *const *handles, int32_t n, int32_t n_steps);

/* A batch of independent simulations stepped as one HIP graph: graph_steps (even, >= 2) steps of
 * every instance are captured once -- a fork from the first instance's stream, each instance's
 * kernels on its own stream, a join back -- and replayed as one launch on the first instance's
 * stream, ordered after work already queued on the instances' streams and before later work on
 * them.  The handles (distinct, each bound to a stream of its own, not timing) stay owned by the
 * caller and must outlive the batch; per instance the result is bit for bit that of pf_lbm_step.
 * The graph is captured again when an instance's step parity differs from that at capture (it
 * was stepped on its own); steps beyond a multiple of graph_steps go through pf_lbm_step_batch.
 * Errors: PF_LBM_EINVAL, PF_LBM_ENOMEM, PF_LBM_EDEVICE (message from pf_lbm_batch_last_error;
 * of pf_lbm_batch_create: pf_lbm_last_error(NULL)). */
typedef struct pf_lbm_batch pf_lbm_batch;
int pf_lbm_batch_create(pf_lbm *const *handles, int32_t n, int32_t graph_steps, pf_lbm_batch **out);
int pf_lbm_batch_step(pf_lbm_batch *b, int32_t n_steps);
void pf_lbm_batch_destroy(pf_lbm_batch *b);
const char *pf_lbm_batch_last_error(const pf_lbm_batch *b);

/* Autotuner of the tile shape of the fluid pass, which leaves the arithmetic unchanged: tiles of
 * 64 x 4 or 64 x 8 nodes (FP64 populations: 64 x 4) marching z-chunks of 4, 8, 16, 32 or 64
 * planes.  Each candidate runs 1 + steps_per_candidate steps of the simulation itself (the state
 * advances), timed with HIP events; the fastest is kept.  out3 (HOST, may be NULL): chosen tile
 * rows, chosen planes per chunk, its mean step time in ms. */
int pf_lbm_autotune(pf_lbm *h, int32_t steps_per_candidate, double *out3);

/* Tile shape of the fluid pass (as pf_lbm_autotune chooses it, or a shape kept from an earlier
 * tuning): tiles of 64 x rows nodes (rows 4 or 8; 4 with FP64 populations) marching z-chunks of
 * planes >= 1 planes.  The arithmetic does not depend on it.  Errors: PF_LBM_EUNSUPPORTED (rows
 * not built for the precision and lattice), PF_LBM_EINVAL. */
int pf_lbm_set_tile(pf_lbm *h, int32_t rows, int32_t planes);

/* Entries of the per-step list of nodes that changed side (Sec. 3.2.2 node conversion) that the
 * handle uses, in [0, 65536] (the default, the list's size in the workspace).  When a step's
 * conversions exceed it, the conversion gather and the closing pass scan the whole bounding box of
 * the phase fields instead of the list; the results are the same.  Lower values exist to run that
 * path on purpose (tests).  Errors: PF_LBM_EINVAL (out of range or NULL handle). */
int pf_lbm_set_event_capacity(pf_lbm *h, int32_t entries);

/* Release the handle (the workspace stays the caller's).  NULL is ignored. */
void pf_lbm_destroy(pf_lbm *h);

/* Message of the last failure on h (or of the last failed pf_lbm_init when h is NULL). */
const char *pf_lbm_last_error(const pf_lbm *h);

#ifdef __cplusplus
}
#endif

#endif /* PF_LBM_H */
