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
 *   Sec. 5.2        heterogeneous worlds (per-world sizes, masks);
 *   Sec. 3, Eq. 2   joint drives (implicit PD, armature, viscous damping)
 *                   as regularised rows (R and v* of the KKT system), and
 *                   the Moreau-Jean midpoint variant of the time step.
 *
 * Conventions.  Quaternions are (x, y, z, w).  Twists are (v, w), w in the
 * world frame.  A joint couples body_a (a body of the same world) and body_b
 * (another body of that world, or -1 for the fixed world); each side carries
 * a frame (position, quaternion) in that body's frame (in the world frame
 * for body_b = -1) whose x axis is the joint axis.  A contact normal points
 * from body_b to body_a; a positive normal impulse separates them.  Constraint
 * rows of a world are ordered: 5 rows per joint (joint order), one row per
 * joint with a limit, one row per joint with an implicit drive (joint
 * order), then 3 rows (n, t1, t2) per contact.
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
typedef struct kamx_mlp_s *kamx_mlp;
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
#define KAMX_WARM_LEARNED 3  /* prediction of the attached network         */

#define KAMX_EULER 0       /* semi-implicit Euler (Sec. 3)                            */
#define KAMX_MOREAU_JEAN 1 /* Moreau-Jean midpoint: constraints, forces and contacts at
                              q + dt/2 u-, then q+ = q_mid + dt/2 u+ (Sec. 3)         */

#define KAMX_SCHED_INDEX 0 /* one launch per step, worlds of a bucket in index order           */
#define KAMX_SCHED_LPT 1   /* one launch per step, by decreasing previous iteration count       */
#define KAMX_SCHED_CHAIN 2 /* multi-step calls keep each world on its workgroup for up to 64
                              steps per launch; single steps as LPT (default)                 */

/* Limits of one world (per-world problem sizes above these are rejected). */
#define KAMX_MAX_BODIES_PER_WORLD 64
#define KAMX_MAX_JOINTS_PER_WORLD 64
#define KAMX_MAX_CONTACTS_PER_WORLD 64
#define KAMX_MAX_ROWS_PER_WORLD 224

/* Limits of a world solved matrix-free (Sec. 5.1: the Delassus operator
 * applied through the Jacobian, Conjugate Residual inner solves).  Rows run
 * one per thread with each contact's three rows in an aligned group of four:
 * align4(5 joints + limits + drives) + 4 * contacts must not exceed
 * KAMX_MAX_THREAD_ROWS_SPARSE. */
#define KAMX_MAX_BODIES_SPARSE 160
#define KAMX_MAX_JOINTS_SPARSE 200
#define KAMX_MAX_THREAD_ROWS_SPARSE 1024

/* Linear solver of Alg. 1 step 5 (Sec. 5.1), chosen per world at model
 * creation.  DENSE: the Delassus matrix is assembled and factored once per
 * step (worlds within the per-world limits above).  SPARSE: matrix-free
 * Delassus products with cr_iters Conjugate Residual iterations per ADMM
 * iteration, warm-started at the previous iterate (worlds within the sparse
 * limits).  AUTO: dense where a world fits the dense limits, else sparse. */
#define KAMX_SOLVER_AUTO 0
#define KAMX_SOLVER_DENSE 1
#define KAMX_SOLVER_SPARSE 2

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
 * gets one unilateral row against the nearer bound.  Gaussian noise of the
 * model's torque_sigma is added along the coordinate c when actuated != 0.
 *
 * Drive.  With implicit_drive = 0, kp and kd act explicitly: the generalized
 * force kp (ref - c) - kd dc/dt from the step's start configuration;
 * damping and armature must then be 0.  With implicit_drive != 0 the joint
 * gets a drive row (Sec. 3: gains absorbed into the constraint rows; Eq. 2:
 * R and v*): over the step the drive's impulse is
 *   dt [kp (ref - c - h dc+/dt) - (kd + damping) dc+/dt
 *       - armature (dc+/dt - dc-/dt) / dt],
 * PD on the coordinate reached at the end of the step, viscous damping on
 * the new rate, and the rotor's reflected inertia (armature, kg m^2 or kg)
 * opposing the change of rate; h is the time from the configuration the
 * row is built at to the end of the step (dt; dt/2 for KAMX_MOREAU_JEAN).
 * The row has R = 1 / (dt K) and v* = -(kp (ref - c) + armature dc-/dt /
 * dt) / K with K = kp h + kd + damping + armature / dt > 0, so it is stable
 * for any gains.  Joints must be sorted by world. */
typedef struct {
    int32_t type;
    int32_t world;
    int32_t body_a, body_b;
    float frame_a[7];
    float frame_b[7];
    float limit_lo, limit_hi;
    float kp, kd, ref;
    int32_t actuated;
    float damping, armature;
    int32_t implicit_drive;
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

/* Box geometry for generated contacts: half extents along the body axes
 * (all zero: the body is not a box) and friction coefficient. */
typedef struct {
    float half[3];
    float mu;
} kamx_box_desc;

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
    int32_t integrator;   /* KAMX_EULER or KAMX_MOREAU_JEAN                   */
    int32_t linear_solver; /* KAMX_SOLVER_*; fixed at model creation          */
    int32_t cr_iters;     /* Conjugate Residual iterations per ADMM iteration
                             (matrix-free worlds; 1..1000)                   */
    /* Adaptive penalty on limit and contact rows (not in the paper, whose
     * penalty is fixed through a solve: residual balancing after Boyd et al.
     * 2011, Sec. 3.4.1).  At iterations adapt_first * 2^j a solve that has
     * not exited compares its residuals: r_d > adapt_ratio r_p divides the
     * limit and contact rows' penalty by adapt_factor, r_p > adapt_ratio r_d
     * multiplies it; a change refactors D~ + diag(eta + rho) (dense worlds)
     * and restarts the acceleration at the current iterate.  The fixed point
     * is unchanged.  adapt_ratio 0 switches it off. */
    float adapt_ratio;
    float adapt_factor;
    int32_t adapt_first;
} kamx_params;

/* Fill *p with defaults (dt 2 ms, gravity -9.81 z, eta 1e-4, rho 1e-4 / 0.3,
 * eps 1e-6, 2000 iterations, acceleration and preconditioning on, restart
 * factor 0.999, beta 0.2, cold start, margin 0.02 m, no noise, semi-implicit
 * Euler, solver chosen by world size, 9 Conjugate Residual iterations,
 * adaptive unilateral penalty with ratio 10 and factor 5 from iteration 100).  Position-level terms act over the time from the configuration
 * the rows are built at to the end of the step: the Baumgarte bias of a
 * bilateral row is beta f / h, a separated contact or limit f / h, a
 * penetrating one beta f / h, with h = dt (Euler) or dt/2 (Moreau-Jean). */
void kamx_default_params(kamx_params *p);

/* Create a model of n_worlds worlds (Sec. 3: the bodies, Eq. 1, and the
 * joints between body pairs or a body and the world that a world's
 * multi-body system is made of; Sec. 5.2: many such worlds, of different
 * structure, in one batch).  bodies[nb], joints[nj], probes[np]
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
 * model: the configuration and generalized velocity of every body (Sec. 3;
 * position + unit quaternion (x, y, z, w), then linear and world-frame
 * angular velocity).  as_reset_state != 0 also stores them as the reset state.
 * Stream-ordered. */
kamx_status kamx_state_upload(kamx_model m, const float *q_dev, const float *u_dev, int32_t as_reset_state,
                              kamx_stream stream);

/* Copy the current poses and twists out to q_dev [nb*7], u_dev [nb*6]: the
 * state the last step advanced to (Sec. 3, the time-stepping scheme). */
kamx_status kamx_state_download(kamx_model m, float *q_dev, float *u_dev, kamx_stream stream);

/* Use explicit contacts for the following steps instead of probes:
 * contacts_dev [n] (device array of kamx_contact, grouped by world in world
 * order, body indices global) and world_offsets [n_worlds+1] (host).  At most
 * max_contacts_per_world contacts per world.  contacts_dev = NULL returns to
 * probe contacts.  The contact array must stay valid while steps using it
 * are pending. */
kamx_status kamx_contacts_upload(kamx_model m, const kamx_contact *contacts_dev, const int32_t *world_offsets,
                                 kamx_stream stream);

/* Generate the contacts of every following step from box geometry
 * (boxes [nb], host; copied): vertex-face tests of every box vertex against
 * a bin made of the floor z = 0 and walls at x = +-half_x, y = +-half_y, and
 * against the faces of every other box of the world (the vertex must lie
 * over the face).  A contact (Sec. 3) has the vertex as its point, the face
 * normal pointing from the face's body (b; -1 for the bin) to the vertex's
 * body (a), the signed distance as gap, friction min(mu_a, mu_b) (the
 * box's own mu against the bin) and key ((target * 64 + box) * 8 + vertex)
 * with targets 0-4 the floor and walls -x, +x, -y, +y and 5 + k the k-th box
 * of the world.  Candidates with gap below margin are kept, the deepest
 * first (ties by key), up to max_contacts_per_world.  At most 20 boxes per
 * world.  Replaces probe and uploaded contacts until kamx_contacts_upload is
 * called; boxes = NULL turns generation off.  When every size bucket holds
 * at least 160 rows, each step kernel generates its world's contacts from
 * the poses the step starts from (and multi-step calls run chained);
 * otherwise a generation kernel runs before every step.  EINVAL on bad
 * geometry or a model without contact capacity. */
kamx_status kamx_contacts_box_bin(kamx_model m, const kamx_box_desc *boxes, float half_x, float half_y,
                                  float margin);

/* External generalized joint forces joint_torque_dev [nj] added to the
 * actuation of every following step (Sec. 3, Eq. 1: part of the generalized
 * forces h of the free velocity); NULL clears them. */
kamx_status kamx_set_external(kamx_model m, const float *joint_torque_dev, kamx_stream stream);

/* Impulses that initialize the solver's iterates (Alg. 1 step 2; Sec. 4.1,
 * warm starting) in KAMX_WARM_EXTERNAL mode:
 * lambda_dev [rows_capacity] in physical units at the row offsets of
 * kamx_model_info.  Copied at the call. */
kamx_status kamx_set_warmstart(kamx_model m, const float *lambda_dev, kamx_stream stream);

/* How steps are mapped onto workgroups (KAMX_SCHED_*).  The mapping decides
 * only which workgroup runs a world's step and when: results are bitwise
 * identical under every mode.  Convergence is uneven (Sec. 4.1; the paper
 * notes the tail effect, Sec. 6.2): ~1% of biped steps need the whole
 * iteration budget.  With one launch per step every step waits for its
 * slowest world; ordering by the previous count (LPT) helps only as far as
 * slow steps recur.  CHAIN keeps each world on one workgroup for a run of
 * steps, so a slow solve delays only its own world and the hardware
 * balances whole chains.  Chains apply to calls of kamx_step with
 * nsteps > 1 unless contacts come from a generation kernel launched before
 * every step (boxes in a bin with buckets below 160 rows); then steps are
 * launched one by one.  Host-side, synchronous; EINVAL on an unknown mode. */
kamx_status kamx_set_schedule(kamx_model m, int32_t mode);

/* Size buckets (Sec. 5.2: worlds of different sizes share one call; each
 * bucket is padded to a row capacity of 32, 64, ..., 224 and runs its own
 * kernel instantiation, largest bucket first).  kamx_bucket_count gives
 * their number.  kamx_bucket_info reports bucket b: its row capacity, its
 * number of worlds, the workgroup size its kernel currently runs with, and
 * the sizes it is built for (n_variants of them, at most 4, written to
 * variants[4] when that is not NULL; the first is the default).  Any
 * output pointer may be NULL.  EINVAL on a bucket index out of range. */
kamx_status kamx_bucket_count(kamx_model m, int32_t *n_buckets);
kamx_status kamx_bucket_info(kamx_model m, int32_t bucket, int32_t *rows_cap, int32_t *n_worlds,
                             int32_t *threads, int32_t *n_variants, int32_t *variants);

/* Workgroup size of bucket b's step kernel: one of its variants.  A smaller
 * workgroup lets more worlds share a compute unit (every kernel keeps two
 * waves per SIMD); a larger one gives each world more threads.  Results are
 * bitwise the same for every variant.  Drops captured graphs.  EINVAL on a
 * bucket out of range or a size the bucket is not built for. */
kamx_status kamx_set_bucket_threads(kamx_model m, int32_t bucket, int32_t threads);

/* Autotuner: for every bucket with more than one variant, time trial_steps
 * steps of that bucket alone (1 to 64; chained when the schedule allows)
 * under each variant, from the model's current state, and keep the fastest.
 * Each trial runs twice and the second run is timed.  The state the steps
 * change (poses, twists, impulse caches, contact keys, statistics, step
 * counter, generated contacts, reset counts) is saved before and restored
 * after every trial, so the model continues exactly as if the call had not
 * been made; an iteration log set by kamx_set_iteration_log is not written.
 * Synchronous (waits for the device); allocates a snapshot of the state for
 * the duration of the call.  ms_out, when not NULL, is a host array
 * [n_buckets * 4] that receives the timed milliseconds of each bucket's
 * variants in kamx_bucket_info order (0 for a bucket with one variant or an
 * unused entry).  EINVAL when trial_steps is outside 1..64. */
kamx_status kamx_autotune(kamx_model m, int32_t trial_steps, float *ms_out);

/* Advance every world by nsteps steps (asynchronous on stream).  nsteps = 1
 * enqueues the step's kernels directly.  nsteps > 1 either runs chained
 * launches (KAMX_SCHED_CHAIN, up to 64 steps per launch) or replays
 * captured graphs of up to 32 single-step launches (the loops that run each
 * world to convergence stay inside the kernels, so the graph has fixed
 * shape, Sec. 5.2); a graph is captured on first use of a step count and
 * reused until a call that changes a kernel argument (kamx_set_params,
 * kamx_set_external, kamx_contacts_upload with another array,
 * kamx_set_schedule, kamx_set_iteration_log, kamx_contacts_box_bin,
 * kamx_model_attach_mlp) drops it.  Results equal nsteps single steps
 * bitwise.  Do not call with nsteps > 1 while the stream is itself being
 * captured (use nsteps = 1 there). */
kamx_status kamx_step(kamx_model m, int32_t nsteps, kamx_stream stream);

/* Iteration count (Alg. 1 iterations run), active row count and status
 * bits (KAMX_WORLD_*) of every step of every following kamx_step call:
 * iters_dev, rows_dev and status_dev [steps][n_worlds] (device,
 * caller-owned, valid while steps are pending; rows_dev and status_dev may
 * be NULL); row k holds the k-th step of the call, steps beyond `steps` are
 * not logged.  iters_dev = NULL turns logging off.  EINVAL if steps < 1. */
kamx_status kamx_set_iteration_log(kamx_model m, int32_t *iters_dev, int32_t *rows_dev, int32_t *status_dev,
                                   int32_t steps);

/* Forward kinematics for resets (Sec. 6.3): move every body of every world
 * so that all joint constraints hold (the passive joints of kinematic loops
 * included) and each joint j with a finite targets_dev[j] (device, [nj],
 * global joint order; NaN = free) sits at that coordinate, keeping each
 * world's reset body where it is (worlds without one move all bodies).
 * Gauss-Newton from the current poses: F = (the five constraint functions
 * of every joint, c_j - target_j), least-change steps -M^-1 J^T (J M^-1 J^T
 * + mu)^-1 F (Jacobi-scaled, mu = 1e-5 on the unit diagonal), bodies moved
 * by the exponential map; F and the poses in FP64, the linear solves in
 * FP32.  Stops when |F|_inf <= tol or after max_iters iterations.  The
 * poses are written back (FP32) and the twists set to zero; iters_dev and
 * resid_dev [n_worlds] (device, may be NULL) receive the iterations taken
 * and |F|_inf at the returned FP64 poses (NaN when the normal matrix could
 * not be factored, or when a world has more than 224 rows with its target
 * rows: 5 per joint plus one per target, that world is left unchanged).
 * Asynchronous on stream; EINVAL on bad arguments. */
kamx_status kamx_forward_kinematics(kamx_model m, const float *targets_dev, int32_t max_iters, float tol,
                                    int32_t *iters_dev, float *resid_dev, kamx_stream stream);

/* The iterate Alg. 1 returns (step 11), for checking the reported
 * residuals (step 9) from outside: every following step writes, for every
 * row r of every world (at the row offsets of kamx_model_info),
 * iterate_dev[4 r .. 4 r + 3] = (x~, y~, z~, p): the last x, y and z of the
 * world's solve in preconditioned units and the row's Jacobi scale
 * (Sec. 4.1), so that lambda = p y~; rows beyond a world's active count get
 * zeros.  iterate_dev (device, [rows_capacity * 4] floats, 16-byte aligned,
 * caller-owned, valid while steps are pending) or NULL (off).  Drops
 * captured graphs; not written by kamx_autotune's trials.  EINVAL when
 * misaligned. */
kamx_status kamx_set_iterate_log(kamx_model m, float *iterate_dev);

/* The constraint impulses the solve returned (Alg. 1 step 11, lambda =
 * P y after un-scaling) for the last step (physical units, N s) into lambda_dev
 * [rows_capacity]; rows beyond a world's active count are zero. */
kamx_status kamx_read_impulses(kamx_model m, float *lambda_dev, kamx_stream stream);

/* Per-world results of the last step (Alg. 1 steps 9-10: the residuals of
 * the exit test and the iteration at which it passed or the budget ran
 * out): iterations iters_dev [n_worlds],
 * residuals resid_dev [n_worlds*4] = (r_p, r_d, r_c, r_ncp) in
 * preconditioned units, status_dev [n_worlds] (KAMX_WORLD_* bits) and the
 * active row count rows_dev [n_worlds].  Any pointer may be NULL. */
kamx_status kamx_read_stats(kamx_model m, int32_t *iters_dev, float *resid_dev, int32_t *status_dev,
                            int32_t *rows_dev, kamx_stream stream);

/* Restart decisions of the last step when log_restarts was set:
 * log_dev [n_worlds * max_iters] bytes, one per iteration: bit 0 = restart
 * of the acceleration (Alg. 1 step 8), bits 1-2 = the adaptive penalty's
 * change at that iteration (1 lowered, 2 raised, 0 none). */
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
 * residuals, updates), entry 14 the index of the compute unit that ran the
 * world and entry 15 its raw hardware id register.  Only available
 * when the environment variable KAMX_PHASE_CLOCK was set at model creation;
 * otherwise ESTATE. */
kamx_status kamx_read_phase_clock(kamx_model m, uint64_t *clk_dev, kamx_stream stream);

/* ---- learned warm start --------------------------------------------------
 * Not in the paper, whose only warm start is the previous step's impulses
 * (Sec. 4.1).  A network predicts a world's dual impulses for the coming
 * step from its state features; the prediction only sets the starting point
 * of Alg. 1 (the exit test on the residuals is unchanged), so a poor
 * prediction costs iterations, never accuracy.
 *
 * Network: x^ = (x - mu_in) / sigma_in; z1 = W1 x^ + b1, h1 = gelu(z1);
 * z2 = W2 h1 + b2, h2 = gelu(z2); y = mu_out + sigma_out (W3 h2 + b3), with
 * gelu the erf form.  Every product runs on the matrix cores with BF16
 * operands (round to nearest even) and FP32 accumulation; master weights,
 * Adam moments and gradients are FP32.  Training minimises the mean squared
 * error of the standardised outputs with bias-corrected Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8).
 *
 * Packed parameter order (FP32, row-major): W1 [n_hidden][n_in_pad],
 * b1 [n_hidden], W2 [n_hidden][n_hidden], b2 [n_hidden],
 * W3 [n_out_pad][n_hidden], b3 [n_out_pad]; n_in_pad and n_out_pad are
 * n_in and n_out rounded up to multiples of 64 (padding entries stay zero
 * under training).  Batches are padded to multiples of 64 inside. */

/* Create a network with initial weights U(-1/sqrt(fan_in), 1/sqrt(fan_in))
 * drawn from splitmix64(seed), identity normalisation, and workspace for
 * batches up to max_batch.  n_hidden must be a multiple of 64 in [64, 4096].
 * EINVAL on bad sizes, ENOMEM when device memory runs out. */
kamx_status kamx_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, uint64_t seed,
                            kamx_mlp *out);
kamx_status kamx_mlp_destroy(kamx_mlp net);

/* Padded sizes and the number of packed FP32 parameters. */
kamx_status kamx_mlp_info(kamx_mlp net, int32_t *n_in_pad, int32_t *n_out_pad, int64_t *n_params);

/* Standardisation of inputs and outputs (device arrays mu_in, sigma_in
 * [n_in], mu_out, sigma_out [n_out]).  An input with sigma <= 1e-12 is
 * ignored (scale 0); an output with sigma <= 1e-12 uses sigma 1. */
kamx_status kamx_mlp_set_normalization(kamx_mlp net, const float *mu_in, const float *sigma_in, const float *mu_out,
                                       const float *sigma_out, kamx_stream stream);

/* y_dev [batch][n_out] = network(x_dev [batch][n_in]); 1 <= batch <= max_batch. */
kamx_status kamx_mlp_forward(kamx_mlp net, const float *x_dev, int32_t batch, float *y_dev, kamx_stream stream);

/* The forward pass of kamx_mlp_forward for callers that cannot allocate
 * device memory (code under stream or graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same kernels, same result bit for bit,
 * but the normalised input and both hidden activations live in a fixed
 * 16 MiB device array that the library holds on every GPU it runs on until
 * the process ends; this call allocates nothing and frees nothing.  x_dev
 * [batch][n_in] and y_dev [batch][n_out] are the caller's device arrays.
 * Limit: pad64(batch) * (n_in_pad + 2 n_hidden) * 2 bytes <= 16 MiB (for
 * 704 padded inputs and 256 hidden units, batch <= 6848); a larger batch is
 * rejected with EINVAL before any work is enqueued.  The network's own
 * max_batch does not apply.  Every call on one GPU shares that GPU's array
 * and overwrites it: calls that overlap on one GPU (on different streams,
 * or with a kamx_mlp_forward_noalloc of another network) race; calls
 * ordered on one stream do not.  EDEVICE if the array's address cannot be
 * obtained. */
kamx_status kamx_mlp_forward_noalloc(kamx_mlp net, const float *x_dev, int32_t batch, float *y_dev,
                                     kamx_stream stream);

/* One Adam step on the mean squared error of the standardised outputs
 * against y_target_dev [batch][n_out] (physical units).  loss_dev (device,
 * may be NULL) receives the loss before the update. */
kamx_status kamx_mlp_train_step(kamx_mlp net, const float *x_dev, const float *y_target_dev, int32_t batch, float lr,
                                float *loss_dev, kamx_stream stream);

/* Packed FP32 parameters: set != 0 copies buf_dev in (and clears the Adam
 * state), set == 0 copies them out. */
kamx_status kamx_mlp_weights(kamx_mlp net, float *buf_dev, int32_t set, kamx_stream stream);

/* Gradients of the last kamx_mlp_train_step (packed order) into buf_dev. */
kamx_status kamx_mlp_gradients(kamx_mlp net, float *buf_dev, kamx_stream stream);

/* Feature and slot sizes of a model whose worlds share one structure (same
 * bodies, joints, limited and driven joints and contact capacity; else
 * EUNSUPPORTED).  Slots: the 5 rows of every joint, the limit rows and the
 * drive rows in row order, then three (n, t1, t2) per contact key 0 ..
 * contact capacity - 1 (the probe index for probe contacts).  Features per
 * world: for every body its position relative to the world's reset body
 * (3), quaternion (4), linear and angular velocity (6) at the configuration
 * the step's rows are built at (the half-step poses for KAMX_MOREAU_JEAN);
 * then the previous step's impulses by slot (zero after a reset); then the
 * explicit generalized joint forces of the coming step (explicit PD, noise
 * and external). */
kamx_status kamx_model_feature_dims(kamx_model m, int32_t *n_features, int32_t *n_slots);

/* Features of the coming step into x_dev [n_worlds][n_features]. */
kamx_status kamx_model_features(kamx_model m, float *x_dev, kamx_stream stream);

/* Impulses of the last step by slot into y_dev [n_worlds][n_slots]
 * (physical units; slots without a contact are zero): the training targets
 * of the network. */
kamx_status kamx_read_impulse_slots(kamx_model m, float *y_dev, kamx_stream stream);

/* Network used by KAMX_WARM_LEARNED: n_in = n_features, n_out = n_slots,
 * batch capacity >= n_worlds; NULL detaches.  The model keeps the pointer
 * (the caller keeps the network alive while steps use it); its weights may
 * change between steps.  With the network attached and warmstart LEARNED,
 * every step of every world evaluates the network inside the step kernel
 * (features as in kamx_model_features, the batched kernels' matrix-core
 * operand layout and accumulation order, so the prediction equals
 * kamx_mlp_forward's bit for bit) and warm starts the solve from the
 * prediction by slot (Alg. 1 step 2 with the previous-step cache replaced
 * by the prediction).  Works in chained launches too. */
kamx_status kamx_model_attach_mlp(kamx_model m, kamx_mlp net);

/* Message of the last failed call on this thread ("" if none). */
const char *kamx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KAMX_H */
