// Internal layouts shared by the HIP kernels and the host runtime of libkamx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kamx.h"

namespace kamx {

constexpr int kMaxBodies = KAMX_MAX_BODIES_PER_WORLD;
constexpr int kMaxJoints = KAMX_MAX_JOINTS_PER_WORLD;
constexpr int kMaxContacts = KAMX_MAX_CONTACTS_PER_WORLD;
constexpr int kMaxRows = KAMX_MAX_ROWS_PER_WORLD;
constexpr int kJointFloats = 24;  // frame_a 7, frame_b 7, lo, hi, kp, kd, ref, damping, armature, pad

// row kinds
constexpr int kRowBilateral = 0;
constexpr int kRowLimit = 1;
constexpr int kRowNormal = 2;
constexpr int kRowTangent = 3;

// joint flag bits (jint[4*j+3])
constexpr int kJointActuated = 1;
constexpr int kJointLimited = 2;
constexpr int kJointDriven = 4;  // implicit drive row (PD, damping, armature)

// Per-world table (one 64-byte record per world).
struct WorldInfo {
    int32_t b0, nb;         // global first body, body count
    int32_t j0, nj;         // global first joint, joint count
    int32_t p0, np;         // global first probe, probe count
    int32_t nlim;           // limited joints
    int32_t row_base;       // first row of the world in row-indexed buffers
    int32_t row_cap;        // row capacity (joint + limit + 3 * contact capacity)
    int32_t contact_cap;    // contact capacity
    int32_t reset_body;     // world-local body index, or -1
    int32_t ndrv;           // joints with an implicit drive row
    int32_t sparse;         // 1: solved matrix-free (Conjugate Residual inner solves)
    int32_t pad[3];
};

struct SolverParams {
    float dt, gx, gy, gz;
    float eta, rho_bil, rho_c, eps;
    int32_t max_iters, fixed_iters, accel;
    float restart_factor;
    int32_t precond;
    float baumgarte;
    int32_t warmstart;
    float contact_margin;
    float torque_sigma;
    uint32_t seed_lo, seed_hi;
    float reset_height;
    int32_t log_restarts;
    int32_t integrator;  // KAMX_EULER or KAMX_MOREAU_JEAN
    int32_t cr_iters;    // Conjugate Residual iterations per x-update (matrix-free worlds)
    float adapt_ratio;   // adaptive unilateral penalty: residual ratio (0: off)
    float adapt_factor;  // factor of one penalty change
    int32_t adapt_first; // first checkpoint iteration (then doubling)
};

// Slot of a contact key in the learned warm start's per-world layout (three
// slots per contact): the key modulo 8 * kMaxBodies -- the probe index for
// probe contacts, box * 8 + vertex for generated box contacts (the target
// the vertex touches is dropped, so a vertex stays in its slot as it slides
// from one face to another), the caller's key modulo 512 otherwise.
__host__ __device__ inline int contact_slot(int key) { return key & (8 * kMaxBodies - 1); }

// Whether iteration it is a checkpoint of the adaptive penalty: first,
// 2 first, 4 first, ...
__host__ __device__ inline bool adapt_checkpoint(int it, int first) {
    if (first <= 0 || it < first || it % first != 0) return false;
    const int q = it / first;
    return (q & (q - 1)) == 0;
}

// A pose advanced by time h with a twist: r + h v, and exp(h [w]x) R by
// the quaternion exponential (left multiplication, world-frame w),
// renormalised.  The end-of-step pose update, and (Moreau-Jean) the
// half-step configuration the rows are built at; evaluated in FP64 there,
// by the step kernel and the contact generation kernel alike, so both see
// the same bits.
template <typename T>
__device__ inline void advance_pose(const T q[7], const T u[6], T h, T out[7]) {
    for (int k = 0; k < 3; ++k) out[k] = q[k] + h * u[k];
    const T wn = sqrt(u[3] * u[3] + u[4] * u[4] + u[5] * u[5]);
    T dq[4] = {T(0), T(0), T(0), T(1)};
    if (wn > T(0)) {
        const T half = T(0.5) * h * wn;
        const T sh = sin(half) / wn;
        dq[0] = u[3] * sh;
        dq[1] = u[4] * sh;
        dq[2] = u[5] * sh;
        dq[3] = cos(half);
    }
    const T *p = q + 3;
    T r[4];
    r[0] = dq[3] * p[0] + dq[0] * p[3] + dq[1] * p[2] - dq[2] * p[1];
    r[1] = dq[3] * p[1] - dq[0] * p[2] + dq[1] * p[3] + dq[2] * p[0];
    r[2] = dq[3] * p[2] + dq[0] * p[1] - dq[1] * p[0] + dq[2] * p[3];
    r[3] = dq[3] * p[3] - dq[0] * p[0] - dq[1] * p[1] - dq[2] * p[2];
    const T nn = T(1) / sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
    for (int k = 0; k < 4; ++k) out[3 + k] = r[k] * nn;
}

// ---- learned warm start: numerics shared by the batched network kernels
// and the per-world inference inside the step kernel, so both produce the
// same bits
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ inline __bf16 to_bf16(float v) { return (__bf16)v; }

// Device view of a network's parameters (BF16 weights row-major
// [out][in_pad], FP32 biases and standardisation).
struct MlpView {
    const __bf16 *w1, *w2, *w3;
    const float *b1, *b2, *b3;
    const float *mu_in, *s_in, *mu_out, *sd_out;
    int32_t n_in, fp, H, n_out, op;
};

struct StepArgs {
    const WorldInfo *worlds;
    const int32_t *bucket_worlds;  // worlds handled by this launch
    int32_t n_bucket_worlds;
    // bodies
    const float *mass;     // [nb]
    const float *inertia;  // [nb*3] principal moments
    float *q;              // [nb*7]
    float *u;              // [nb*6]
    const float *q0;       // reset state
    const float *u0;
    // joints
    const int32_t *jint;   // [nj*4]: type, local a, local b (-1 world), flags
    const float *jf;       // [nj*kJointFloats]
    const float *ext_tau;  // [nj] or null
    // probes
    const int32_t *pbody;  // [np] local body
    const float *pf;       // [np*4]: point, mu
    // explicit contacts
    const float *box_geom;         // non-null: contacts generated in the step (boxes in a bin)
    float bin_wx, bin_wy, bin_margin;
    const kamx_contact *contacts;  // null: use probes
    const int32_t *coff;           // [n_worlds+1]
    const int32_t *ccount;         // non-null: contacts of world w at w * kMaxContacts, ccount[w] of them
    // outputs and caches
    float *lambda;          // [rows] impulses of the last step (physical)
    const float *lambda_ext;  // [rows] external warm start
    int32_t *keys;          // [n_worlds*kMaxContacts] contact keys of the last step
    int32_t *iters;
    float *resid;           // [n_worlds*4]
    int32_t *status;
    int32_t *rows;          // active rows per world
    uint8_t *rlog;          // [n_worlds*max_iters] or null
    float *iterate_out;     // [rows*4] final (x~, y~, z~, p) per row, or null
    float *tau_out;         // [nj]
    kamx_contact *contacts_out;  // [n_worlds*kMaxContacts]
    int32_t *ncontacts_out;      // [n_worlds]
    int32_t *reset_count;        // [n_worlds]
    uint64_t *phase_clk;         // [n_worlds*16] phase time stamps, or null
    SolverParams p;
    const uint32_t *step_ctr;    // device step counter (noise key) at the launch's first step
    int32_t nsteps;              // steps per launch (each workgroup keeps its world for all of them)
    int32_t n_worlds;            // worlds of the model (stride of iter_log)
    int32_t *iter_log;           // [iter_log_rows * n_worlds] iterations of every step, or null
    int32_t *row_log;            // [iter_log_rows * n_worlds] active rows of every step, or null
    int32_t *status_log;         // [iter_log_rows * n_worlds] status bits of every step, or null
    int32_t iter_log_rows;       // steps of this launch that have a log row
    // learned warm start
    int32_t stage;               // 0: full step; 1: write the features of the coming step and stop
    float *features;             // [n_worlds * n_feat] (stage 1)
    int32_t n_feat;
    float *ws_slots;             // network output [n_worlds * slots] (warm start mode LEARNED)
    MlpView mlp;                 // the network, run inside the step for warm start mode LEARNED
    int32_t n_contact_slots;     // contact keys with a slot (probes per world, else contact capacity)
};

// Packed lower-triangular storage with every row padded to a multiple of 4
// floats (so rows can be read as float4): offset of row i.
__host__ __device__ inline int tri_row_offset(int i) {
    int a = i >> 2, b = i & 3;
    return 4 * (a + 1) * (2 * a + b);
}

// Shared-memory footprint (floats) of the fused step kernel for a row bucket.
__host__ __device__ inline int body_floats() { return 32 * kMaxBodies; }
__host__ __device__ inline int joint_floats() { return 16 * kMaxJoints; }  // tau, Jc[12], a, b, type|flags
__host__ __device__ inline int contact_floats() { return 12 * kMaxContacts; }  // point, normal, gap, mu, a, b, key, slot
__host__ __device__ inline int row_floats(int mc) { return 18 * mc; }
__host__ __device__ inline int vec_floats(int mc) { return 15 * mc; }
__host__ __device__ inline int bodyw_floats() { return 2 * 6 * kMaxBodies; }  // FP64 [6][kMaxBodies]
__host__ __device__ inline int posed_floats() { return 2 * 7 * kMaxBodies; }  // FP64 poses [7][kMaxBodies]
__host__ __device__ inline int inc_floats(int mc) { return ((kMaxBodies + 1 + 2 * mc) + 3) & ~3; }
__host__ __device__ inline int smem_floats(int mc) {
    return body_floats() + joint_floats() + contact_floats() + row_floats(mc) + vec_floats(mc) +
           tri_row_offset(mc) + 64 + bodyw_floats() + posed_floats() + inc_floats(mc);
}

}  // namespace kamx
