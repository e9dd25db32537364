/*
 * kamx.h -- C ABI of the batched constrained-dynamics step on MI355X (gfx950).
 *
 * The library advances many independent maximal-coordinate rigid multi-body
 * worlds by one (or several) time steps of the method of "Kamino: GPU-based
 * Massively Parallel Simulation of Multi-Body Systems with Challenging
 * Topologies" (Tsounis et al., 2026):
 *   Sec. 3, Eq. 1   bodies with SE(3) poses, block-diagonal mass matrix and
 *                   Newton-Euler forces (gravity, gyroscopic, actuation);
 *   Sec. 3          bilateral joint constraints (loops need no special
 *                   treatment), unilateral joint limits, frictional contacts
 *                   on the Coulomb cone, Baumgarte bias, semi-implicit Euler
 *                   with the SO(3) exponential map;
 *   Sec. 4, Eq. 3-4 the dual problem in the constraint impulses with the
 *                   Delassus matrix D = J M^-1 J^T and free velocity v_f;
 *   Sec. 4, Alg. 1  Proximal-ADMM with De Saxce correction, factoring
 *                   D + diag(eta + rho) once per step;
 *   Sec. 4.1        Nesterov acceleration with restart, warm start,
 *                   Jacobi preconditioning, infinity-norm residuals;
 *   Sec. 5.2        heterogeneous worlds (per-world sizes, masks).
 *
 * Conventions.  Quaternions are (x, y, z, w).  Twists are (v, w), w in the
 * world frame.  A joint couples body_a (a body of the same world) and body_b
 * (another body of that world, or -1 for the fixed world); each side carries
 * a frame (position, quaternion) in that body's frame (in the world frame
 * for body_b = -1) whose x axis is the joint axis.  A contact normal points
 * from body_b to body_a; a positive normal impulse separates them.  Constraint
 * rows of a world are ordered: 5 rows per joint (joint order), one row per
 * joint with a limit, then 3 rows (n, t1, t2) per contact.
 *
 * Ownership.  All pointer arguments are owned by the caller.  Arguments named
 * "_dev" are device pointers (e.g. torch tensors' data_ptr()); the rest are
 * host pointers.  Device arrays must stay valid until the work enqueued on
 * the given stream has completed; the library keeps no caller pointer beyond
 * that, except the explicit contact array set by kamx_contacts_upload, which
 * must stay valid while steps that use it are pending.
 *
 * Errors.  Every call returns KAMX_OK or a negative status and records a
 * message readable with kamx_last_error() (per thread).  Argument errors are
 * detected synchronously; asynchronous device faults surface at the next call
 * as KAMX_EDEVICE.  Numerical outcomes of individual worlds (iteration cap,
 * non-finite values, a non-positive pivot) are data in the per-world status
 * array, never call errors.  A model is not thread-safe; distinct models on
 * distinct streams are independent.
 */
#ifndef KAMX_H
#define KAMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kamx_model_s *kamx_model;
typedef struct ihipStream_t *kamx_stream; /* a hipStream_t; NULL = default stream */
typedef int32_t kamx_status;

#define KAMX_OK 0
#define KAMX_EINVAL (-1)
#define KAMX_ENOMEM (-2)
#define KAMX_EDEVICE (-3)
#define KAMX_ESTATE (-4)
#define KAMX_EUNSUPPORTED (-5)

/* per-world status bits (data, not call errors) */
#define KAMX_WORLD_OK 0
#define KAMX_WORLD_MAXITER 1     /* residuals not below eps within max_iters */
#define KAMX_WORLD_NONFINITE 2   /* a non-finite residual stopped the solve  */
#define KAMX_WORLD_FACTOR_FAIL 4 /* non-positive pivot: impulses set to zero */

#define KAMX_REVOLUTE 0
#define KAMX_PRISMATIC 1

#define KAMX_WARM_COLD 0     /* x = y = z = 0                            */
#define KAMX_WARM_PREVIOUS 1 /* previous step's impulses, matched by slot */
#define KAMX_WARM_EXTERNAL 2 /* impulses given by kamx_set_warmstart      */

/* Limits of one world (per-world problem sizes above these are rejected). */
#define KAMX_MAX_BODIES_PER_WORLD 64
#define KAMX_MAX_JOINTS_PER_WORLD 64
#define KAMX_MAX_CONTACTS_PER_WORLD 64
#define KAMX_MAX_ROWS_PER_WORLD 224

/* A rigid body (Sec. 3, Eq. 1): mass and principal moments of inertia in
 * its body frame.  Bodies must be sorted by world. */
typedef struct {
    int32_t world;
    float mass;
    float inertia[3];
} kamx_body_desc;

/* A joint (Sec. 3).  body_a / body_b are global body indices (body_b may be
 * -1).  limit_lo / limit_hi bound the joint coordinate (revolute: angle of
 * A's frame about the axis relative to B's; prismatic: offset of A's anchor
 * along B's axis); NaN means unbounded, and a joint with any finite bound
 * gets one unilateral row against the nearer bound.  Actuation adds the
 * generalized force kp (ref - c) - kd dc/dt along the coordinate c, plus
 * Gaussian noise of the model's torque_sigma when actuated != 0.  Joints must
 * be sorted by world. */
typedef struct {
    int32_t type;
    int32_t world;
    int32_t body_a, body_b;
    float frame_a[7];
    float frame_b[7];
    float limit_lo, limit_hi;
    float kp, kd, ref;
    int32_t actuated;
} kamx_joint_desc;

/* A contact probe: a point fixed in a body, tested each step against the
 * ground plane z = 0; it becomes a contact with normal +z and gap equal to
 * its height when that height is below the model's contact_margin.
 * Probes must be sorted by world. */
typedef struct {
    int32_t world;
    int32_t body;
    float point[3];
    float mu;
} kamx_probe_desc;

/* An explicit contact (Sec. 3): world point, unit normal from b to a, gap
 * (signed distance, negative when penetrating), friction coefficient and a
 * caller key.  body_a is a global body index, body_b a global index or -1. */
typedef struct {
    int32_t body_a, body_b;
    float point[3];
    float normal[3];
    float gap;
    float mu;
    int32_t key;
} kamx_contact;

/* Solver and step parameters (Alg. 1, Sec. 4.1). */
typedef struct {
    float dt;
    float gravity[3];
    float eta;            /* proximal parameter                               */
    float rho_bilateral;  /* ADMM penalty on bilateral rows                   */
    float rho_contact;    /* ADMM penalty on limit and contact rows           */
    float eps;            /* infinity-norm tolerance of the three residuals   */
    int32_t max_iters;    /* iteration cap                                    */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations, no exit   */
    int32_t accel;        /* Nesterov acceleration with adaptive restart      */
    float restart_factor; /* restart when the combined residual does not drop
                             below this factor times the previous one        */
    int32_t precond;      /* Jacobi preconditioning                           */
    float baumgarte;      /* Baumgarte factor beta                            */
    int32_t warmstart;    /* KAMX_WARM_*                                      */
    float contact_margin; /* probe activation distance                        */
    float torque_sigma;   /* std. dev. of actuation noise (N m or N)          */
    uint64_t seed;        /* key of the counter-based noise generator         */
    float reset_height;   /* a world whose reset body is below this height is
                             reset to the stored initial state at step start */
    int32_t log_restarts; /* 1: record the restart decision of every iteration */
} kamx_params;

/* Fill *p with defaults (dt 2 ms, gravity -9.81 z, eta 1e-4, rho 1e-4 / 0.3,
 * eps 1e-6, 2000 iterations, acceleration and preconditioning on, restart
 * factor 0.999, beta 0.2, cold start, margin 0.02 m, no noise). */
void kamx_default_params(kamx_params *p);

/* Create a model of n_worlds worlds.  bodies[nb], joints[nj], probes[np]
 * (np may be 0) are host arrays.  reset_body[n_worlds] (host, may be NULL)
 * names the global body whose height triggers a reset, or -1.  Explicit
 * contacts may later be supplied with up to max_contacts_per_world per world
 * (0: probes only).  Allocates all internal device buffers on the current
 * device and assigns worlds to size buckets by their row capacity.
 * Errors: EINVAL (sizes, sorting, indices, a world above the limits),
 * ENOMEM, EDEVICE. */
kamx_status kamx_model_create(const kamx_body_desc *bodies, int32_t nb, const kamx_joint_desc *joints,
                              int32_t nj, const kamx_probe_desc *probes, int32_t np, const int32_t *reset_body,
                              int32_t n_worlds, int32_t max_contacts_per_world, const kamx_params *params,
                              kamx_model *out);

/* Release the model and its device buffers (synchronizes the device). */
kamx_status kamx_model_destroy(kamx_model m);

/* Replace the parameters (host struct). */
kamx_status kamx_set_params(kamx_model m, const kamx_params *params);

/* Shapes: total bodies, joints, row capacity over all worlds, number of
 * buckets, and the per-world row offsets (host array [n_worlds+1], may be
 * NULL) that index kamx_read_impulses / kamx_set_warmstart buffers. */
kamx_status kamx_model_info(kamx_model m, int32_t *n_bodies, int32_t *n_joints, int32_t *rows_capacity,
                            int32_t *n_buckets, int32_t *row_offsets);

/* Copy poses q_dev [nb*7] and twists u_dev [nb*6] (FP32, device) into the
 * model.  as_reset_state != 0 also stores them as the reset state.
 * Stream-ordered. */
kamx_status kamx_state_upload(kamx_model m, const float *q_dev, const float *u_dev, int32_t as_reset_state,
                              kamx_stream stream);

/* Copy the current poses and twists out to q_dev [nb*7], u_dev [nb*6]. */
kamx_status kamx_state_download(kamx_model m, float *q_dev, float *u_dev, kamx_stream stream);

/* Use explicit contacts for the following steps instead of probes:
 * contacts_dev [n] (device array of kamx_contact, grouped by world in world
 * order, body indices global) and world_offsets [n_worlds+1] (host).  At most
 * max_contacts_per_world contacts per world.  contacts_dev = NULL returns to
 * probe contacts.  The contact array must stay valid while steps using it
 * are pending. */
kamx_status kamx_contacts_upload(kamx_model m, const kamx_contact *contacts_dev, const int32_t *world_offsets,
                                 kamx_stream stream);

/* External generalized joint forces joint_torque_dev [nj] added to the
 * actuation of every following step; NULL clears them. */
kamx_status kamx_set_external(kamx_model m, const float *joint_torque_dev, kamx_stream stream);

/* Impulses used as the warm start in KAMX_WARM_EXTERNAL mode:
 * lambda_dev [rows_capacity] in physical units at the row offsets of
 * kamx_model_info.  Copied at the call. */
kamx_status kamx_set_warmstart(kamx_model m, const float *lambda_dev, kamx_stream stream);

/* Advance every world by nsteps steps (asynchronous on stream). */
kamx_status kamx_step(kamx_model m, int32_t nsteps, kamx_stream stream);

/* Impulses of the last step (physical units, N s) into lambda_dev
 * [rows_capacity]; rows beyond a world's active count are zero. */
kamx_status kamx_read_impulses(kamx_model m, float *lambda_dev, kamx_stream stream);

/* Per-world results of the last step: iterations iters_dev [n_worlds],
 * residuals resid_dev [n_worlds*4] = (r_p, r_d, r_c, r_ncp) in
 * preconditioned units, status_dev [n_worlds] (KAMX_WORLD_* bits) and the
 * active row count rows_dev [n_worlds].  Any pointer may be NULL. */
kamx_status kamx_read_stats(kamx_model m, int32_t *iters_dev, float *resid_dev, int32_t *status_dev,
                            int32_t *rows_dev, kamx_stream stream);

/* Restart decisions of the last step when log_restarts was set:
 * log_dev [n_worlds * max_iters] bytes (1 = restart at that iteration). */
kamx_status kamx_read_restart_log(kamx_model m, uint8_t *log_dev, kamx_stream stream);

/* Generalized joint forces applied in the last step (actuation, noise and
 * external) into torque_dev [nj]. */
kamx_status kamx_read_torques(kamx_model m, float *torque_dev, kamx_stream stream);

/* Contacts used in the last step: contacts_dev [n_worlds *
 * KAMX_MAX_CONTACTS_PER_WORLD] (slot k of world w at w*64 + k) and counts_dev
 * [n_worlds]. */
kamx_status kamx_read_contacts(kamx_model m, kamx_contact *contacts_dev, int32_t *counts_dev, kamx_stream stream);

/* Number of resets performed so far (summed over worlds) into *count (host;
 * synchronizes the stream). */
kamx_status kamx_reset_count(kamx_model m, int64_t *count, kamx_stream stream);

/* Diagnostic: wall-clock stamps (device ticks) of the last step of every
 * world into clk_dev [n_worlds*16]: entries 0-7 at the phase boundaries
 * (start, Delassus, warm start, factor, inverse, iterations, outputs, end),
 * entries 8-13 the ticks spent in the iteration sub-phases (right-hand side,
 * forward mat-vec, transposed mat-vec, body gather, projections and
 * residuals, updates).  Only available
 * when the environment variable KAMX_PHASE_CLOCK was set at model creation;
 * otherwise ESTATE. */
kamx_status kamx_read_phase_clock(kamx_model m, uint64_t *clk_dev, kamx_stream stream);

/* Message of the last failed call on this thread ("" if none). */
const char *kamx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KAMX_H */
