// Fused per-world time step on gfx950: one workgroup advances one world.
//
// Everything a world needs -- body state, joint frames, contact rows, the
// preconditioned Delassus matrix, its factor and the ADMM vectors -- lives in
// LDS for the whole step, so HBM sees only the per-world inputs and outputs.
// Thread i owns constraint row i (and the block that starts at row i: one
// row for joints and limits, three rows for a contact).
//
// Steps (Tsounis et al. 2026):
//   bodies: R(q), M^-1 applied in the body frame, Newton-Euler forces with
//           gyroscopic term and joint actuation (Sec. 3, Eq. 1);
//   rows:   joint / limit / contact Jacobians and Baumgarte bias (Sec. 3);
//   D~:     D = J M^-1 J^T (Eq. 4) scaled by the Jacobi preconditioner
//           (Sec. 4.1), shifted by eta + rho (Alg. 1 step 1);
//   factor: Cholesky once per step, then the explicit inverse of the factor,
//           so every iteration's solve is two parallel triangular mat-vecs
//           instead of two serial substitution sweeps;
//   PADMM:  Alg. 1 steps 4-10 with Nesterov restart (Sec. 4.1);
//   output: lambda = P y, u+ = u_f + M^-1 J^T lambda, SO(3) exponential map.
#include <math.h>

#include "kamx_boxbin.h"
#include "kamx_device.h"
#include "kamx_geom.h"
#include "kamx_internal.h"

namespace kamx {

// ---------------------------------------------------------------------------
// LDS views
// ---------------------------------------------------------------------------

// body fields [field][kMaxBodies]
enum { BQ = 0, BU = 7, BUF = 13, BR = 19, BII = 28, BIM = 31 };
// joint fields [field][kMaxJoints]
enum { JTAU = 0, JC = 1, JA = 13, JB = 14, JTF = 15 };
// contact fields [field][kMaxContacts]
enum { CP = 0, CN = 3, CGAP = 6, CMU = 7, CA = 8, CB = 9, CKEY = 10 };
// row fields [field][MC]
enum { RJ = 0, RBIAS = 12, RMU = 13, RIA = 14, RIB = 15, RKIND = 16, RREG = 17 };
// vector fields [field][MC]
enum { VP = 0, VRHO, VVT, VX, VYH, VZH, VYP, VZP, VRHS, VT, VXN, VWS, VAUX, VCOL, VDX };

struct Lds {
    float *b, *j, *c, *r, *v, *A, *red;
    double *wb;          // [6][kMaxBodies] FP64 body work vector
    double *qd;          // [7][kMaxBodies] FP64 poses the rows are built at
    int *inc_off;        // [kMaxBodies + 1] body -> row incidence offsets
    int *inc_list;       // [2 * MC] (row << 1) | side
    int mc;
    __device__ float &bf(int f, int i) const { return b[f * kMaxBodies + i]; }
    __device__ float &jfld(int f, int i) const { return j[f * kMaxJoints + i]; }
    __device__ float &cf(int f, int i) const { return c[f * kMaxContacts + i]; }
    __device__ float &rf(int f, int i) const { return r[f * mc + i]; }
    __device__ int &ri(int f, int i) const { return reinterpret_cast<int *>(r)[f * mc + i]; }
    __device__ float *vec(int f) const { return v + f * mc; }
};

// world-frame rotation of a body (from LDS)
__device__ inline void body_rot(const Lds &L, int b, float R[9]) {
    for (int k = 0; k < 9; ++k) R[k] = L.bf(BR + k, b);
}

// o = M_b^-1 [lin; ang], applied in the body frame: lin / m, R (I^-1 (R^T ang))
__device__ inline void apply_minv(const Lds &L, int b, const float in[6], float out[6]) {
    float im = L.bf(BIM, b);
    out[0] = in[0] * im;
    out[1] = in[1] * im;
    out[2] = in[2] * im;
    float R[9], t[3], s[3];
    body_rot(L, b, R);
    mtv3(R, in + 3, t);
    t[0] *= L.bf(BII + 0, b);
    t[1] *= L.bf(BII + 1, b);
    t[2] *= L.bf(BII + 2, b);
    mv3(R, t, s);
    out[3] = s[0];
    out[4] = s[1];
    out[5] = s[2];
}

// Joint geometry: anchors, lever arms and frame rotations of both sides.
// Evaluated in FP64: the Baumgarte bias multiplies the position-level
// constraint value by beta / dt, so FP32 rounding of near-cancelling anchor
// offsets and near-orthogonal axis products (about 1e-7 absolute) would
// become velocity errors of order 1e-5.  J and everything downstream stay
// FP32.
__device__ inline void joint_geo(const Lds &L, const float *jf, int la, int lb, JointGeo &g) {
    double qa[7], qb[7];
    for (int k = 0; k < 7; ++k) qa[k] = L.qd[k * kMaxBodies + la];
    for (int k = 0; k < 7; ++k) qb[k] = lb >= 0 ? L.qd[k * kMaxBodies + lb] : 0.0;
    joint_geo_q(qa, qb, lb >= 0, jf, g);
}

__device__ inline void put_row(const Lds &L, int r, const float Ja[6], int la, const float Jb[6], int lb, float f,
                               int kind, float mu, const SolverParams &P) {
    for (int k = 0; k < 6; ++k) {
        L.rf(RJ + k, r) = Ja[k];
        L.rf(RJ + 6 + k, r) = lb >= 0 ? Jb[k] : 0.f;
    }
    L.ri(RIA, r) = la;
    L.ri(RIB, r) = lb;
    L.ri(RKIND, r) = kind;
    L.rf(RMU, r) = mu;
    L.rf(RREG, r) = 0.f;
    // position-level terms act over the time from the rows' configuration to
    // the end of the step: dt, or dt / 2 from the Moreau-Jean half step
    float bias = 0.f;
    float inv_h = (P.integrator == KAMX_MOREAU_JEAN ? 2.f : 1.f) / P.dt;
    if (kind == kRowBilateral) bias = P.baumgarte * f * inv_h;
    else if (kind == kRowLimit || kind == kRowNormal) bias = (f >= 0.f ? f : P.baumgarte * f) * inv_h;
    L.rf(RBIAS, r) = bias;
}

// Rows of joint j (5 rows from r0), Sec. 3 bilateral constraints; geometry
// and constraint values in FP64, rows stored in FP32.
__device__ inline void put_row6(const Lds &L, int r, const double Ja[6], int la, const double Jb[6], int lb, double f,
                                int kind, const SolverParams &P) {
    float fa[6], fb[6];
    for (int k = 0; k < 6; ++k) {
        fa[k] = (float)Ja[k];
        fb[k] = (float)Jb[k];
    }
    put_row(L, r, fa, la, fb, lb, (float)f, kind, 0.f, P);
}

__device__ inline void joint_rows(const Lds &L, int type, const JointGeo &g, int la, int lb, int r0,
                                  const SolverParams &P) {
    joint_constraints(type, g, [&](int e, const double Ja[6], const double Jb[6], double f) {
        put_row6(L, r0 + e, Ja, la, Jb, lb, f, kRowBilateral, P);
    });
}

// ---------------------------------------------------------------------------
// block-wide reductions (fixed order: butterfly within a wave, then waves in
// index order), results uniform across the workgroup
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// matrix-free preconditioned Delassus product out = P J M^-1 J^T P x (Eq. 4),
// accumulated in FP64 over the two 6-blocks of every row: bodies gather
// their incident rows (fixed row order), rows then read their two bodies.
// Costs O(rows) instead of O(rows^2); used for the refinement residual of
// every x-update and for the dual residual.
// ---------------------------------------------------------------------------

template <int NT>
__device__ inline void reduce4(float &m0, float &m1, float &m2, float &s3, float *red) {
    // rows of 16 lanes by DPP, then the wave's four rows through readlane,
    // then the waves in order through LDS; every step combines two values
    // that the partner combines in the other order, so all lanes agree.
    // m0, m1, m2 are +0 or above, or NaN (maxima of absolute values)
    m0 = lane_group_max<16>(m0);
    m1 = lane_group_max<16>(m1);
    m2 = lane_group_max<16>(m2);
    s3 = lane_group_sum<16>(s3);
    m0 = max_nonneg(max_nonneg(rdlane(m0, 0), rdlane(m0, 16)), max_nonneg(rdlane(m0, 32), rdlane(m0, 48)));
    m1 = max_nonneg(max_nonneg(rdlane(m1, 0), rdlane(m1, 16)), max_nonneg(rdlane(m1, 32), rdlane(m1, 48)));
    m2 = max_nonneg(max_nonneg(rdlane(m2, 0), rdlane(m2, 16)), max_nonneg(rdlane(m2, 32), rdlane(m2, 48)));
    s3 = (rdlane(s3, 0) + rdlane(s3, 16)) + (rdlane(s3, 32) + rdlane(s3, 48));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[4 * wave + 0] = m0;
        red[4 * wave + 1] = m1;
        red[4 * wave + 2] = m2;
        red[4 * wave + 3] = s3;
    }
    __syncthreads();
    m0 = red[0];
    m1 = red[1];
    m2 = red[2];
    s3 = red[3];
    for (int k = 1; k < NT / 64; ++k) {
        m0 = max_nonneg(m0, red[4 * k]);
        m1 = max_nonneg(m1, red[4 * k + 1]);
        m2 = max_nonneg(m2, red[4 * k + 2]);
        s3 = s3 + red[4 * k + 3];
    }
}

__device__ inline float dot4(const float *a, const float *b) {
    float4 x = *reinterpret_cast<const float4 *>(a);
    float4 y = *reinterpret_cast<const float4 *>(b);
    return x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
}

// ---- 16x16 tiles of the packed lower triangle on the matrix cores
// v_mfma_f32_16x16x4f32: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of a 16x4 by 4x16 product and holds rows
// 4 (l / 16) + c, column l % 16 of the 16x16 accumulator.
typedef float mfx4 __attribute__((ext_vector_type(4)));

__device__ inline mfx4 mfma4(float a, float b, mfx4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

// element (r, c) of the packed lower triangle; 0 above the diagonal
// Workgroup sizes each dense row bucket is built for (the first is the
// default; see step_threads_variants).
struct BucketSizes {
    int mc, n, nt[3];
};
constexpr BucketSizes kBucketSizes[] = {{32, 3, {256, 128, 64}}, {64, 2, {256, 128, 0}}, {96, 2, {512, 256, 0}},
                                        {128, 2, {512, 256, 0}}, {160, 2, {384, 512, 0}}, {192, 2, {384, 512, 0}},
                                        {224, 1, {512, 0, 0}}};

// The default workgroup size of a bucket.  The gather's four-thread bodies
// are capped by it rather than by the launched size, so that every size of a
// bucket sums each body in the same order (a smaller size runs the gather's
// tasks in more than one pass).
constexpr int default_bucket_threads(int mc) {
    for (const BucketSizes &v : kBucketSizes)
        if (v.mc == mc) return v.nt[0];
    return 0;
}

__device__ inline float tri_at(const float *A, int r, int c) { return c <= r ? A[tri_row_offset(r) + c] : 0.f; }

// Body gather of the matrix-free product: g_b = sum over the rows incident
// to body b of J_{r,b}^T p_r x_r, one thread per (body, component), FP64,
// rows in increasing order.  Ends with a barrier.
template <int NT>
__device__ inline void delassus_gather(const Lds &L, int nb, const float *vp, const float *x) {
    // two adjacent threads per (body, component) take alternate rows of the
    // incidence list; their partial sums meet by one shuffle
    const int tid = threadIdx.x;
    const int ntask = 12 * nb;
    for (int t0 = 0; t0 < ntask; t0 += NT) {
        const int t = t0 + tid;
        const int bc = t >> 1, h = t & 1;
        const int b = bc / 6, c = bc - 6 * (bc / 6);
        double g0 = 0.0, g1 = 0.0;
        if (t < ntask) {
            int k = L.inc_off[b] + h;
            const int k1 = L.inc_off[b + 1];
            for (; k + 2 < k1; k += 4) {
                int e0 = L.inc_list[k], e1 = L.inc_list[k + 2];
                int r0 = e0 >> 1, r1 = e1 >> 1;
                g0 += (double)L.rf(RJ + 6 * (e0 & 1) + c, r0) * ((double)vp[r0] * (double)x[r0]);
                g1 += (double)L.rf(RJ + 6 * (e1 & 1) + c, r1) * ((double)vp[r1] * (double)x[r1]);
            }
            if (k < k1) {
                int e0 = L.inc_list[k];
                int r0 = e0 >> 1;
                g0 += (double)L.rf(RJ + 6 * (e0 & 1) + c, r0) * ((double)vp[r0] * (double)x[r0]);
            }
        }
        // partner lane (t ^ 1) is the DPP neighbour in the same wave
        const double gs = lane_group_sum<2>(g0 + g1);
        if (t < ntask && h == 0) L.wb[c * kMaxBodies + b] = gs;
    }
    __syncthreads();
}

// The gather with the bodies balanced over the threads: bodies with long
// incidence lists take four threads per component, the others two, so every
// thread walks about the same number of rows. gorder[0] = nh, the count of
// four-thread bodies (passed as nh), and gorder[1..nb] the bodies in task
// order, those nh first. The 12 (nb + nh) tasks run in passes of NT (one
// pass when they fit); a pass starts at a multiple of NT, so the lanes of a
// body's component form an aligned group of 4 or 2 within one wave.
template <int NT>
__device__ inline void delassus_gather_bal(const Lds &L, int nb, int nh, const unsigned char *gorder,
                                           const float *vp, const float *x) {
    const int nheavy = 24 * nh, ntask = nheavy + 12 * (nb - nh);
    // one task per thread; the first pass is straight-line code, the rest
    // (only when the tasks outnumber the threads) loops
    auto task = [&](const int t) {
        const bool heavy = t < nheavy;
        int j, c, h, S;
        if (heavy) {
            j = t / 24;
            const int r = t - 24 * j;
            c = r >> 2;
            h = r & 3;
            S = 4;
        } else {
            const int u = t - nheavy, q = u / 12, r = u - 12 * q;
            j = nh + q;
            c = r >> 1;
            h = r & 1;
            S = 2;
        }
        double g0 = 0.0, g1 = 0.0;
        int b = 0;
        if (t < ntask) {
            b = gorder[1 + j];
            int k = L.inc_off[b] + h;
            const int k1 = L.inc_off[b + 1];
            for (; k + S < k1; k += 2 * S) {
                int e0 = L.inc_list[k], e1 = L.inc_list[k + S];
                int r0 = e0 >> 1, r1 = e1 >> 1;
                g0 += (double)L.rf(RJ + 6 * (e0 & 1) + c, r0) * ((double)vp[r0] * (double)x[r0]);
                g1 += (double)L.rf(RJ + 6 * (e1 & 1) + c, r1) * ((double)vp[r1] * (double)x[r1]);
            }
            if (k < k1) {
                int e0 = L.inc_list[k];
                int r0 = e0 >> 1;
                g0 += (double)L.rf(RJ + 6 * (e0 & 1) + c, r0) * ((double)vp[r0] * (double)x[r0]);
            }
        }
        double gs = g0 + g1;
        gs += dpp<kDppXor1>(gs);
        const double g4 = gs + dpp<kDppXor2>(gs);
        if (t < ntask && h == 0) L.wb[c * kMaxBodies + b] = heavy ? g4 : gs;
    };
    task(threadIdx.x);
    for (int t0 = NT; t0 < ntask; t0 += NT) task(t0 + threadIdx.x);
    __syncthreads();
}

// w = M_b^-1 g_b in FP64 (body frame: R diag(I^-1) R^T for the angular part)
// (the angular part from the body's symmetric R diag(I^-1) R^T, formed once
// per step in FP64 by body_angular_minv)
__device__ inline void body_minv64(const Lds &L, int b, double w[6]) {
    const double *mi = reinterpret_cast<const double *>(L.b);
    double g[6];
    for (int c = 0; c < 6; ++c) g[c] = L.wb[c * kMaxBodies + b];
    const double im = L.bf(BIM, b);
    const double m00 = mi[b], m11 = mi[kMaxBodies + b], m22 = mi[2 * kMaxBodies + b];
    const double m01 = mi[3 * kMaxBodies + b], m02 = mi[4 * kMaxBodies + b], m12 = mi[5 * kMaxBodies + b];
    for (int c = 0; c < 3; ++c) w[c] = g[c] * im;
    // explicit fused multiply-adds: every workgroup-size variant computes the same bits
    w[3] = __builtin_fma(m02, g[5], __builtin_fma(m01, g[4], m00 * g[3]));
    w[4] = __builtin_fma(m12, g[5], __builtin_fma(m11, g[4], m01 * g[3]));
    w[5] = __builtin_fma(m22, g[5], __builtin_fma(m12, g[4], m02 * g[3]));
}

// The angular inverse inertia R diag(I^-1) R^T of every body in FP64 (six
// entries: 00, 11, 22, 01, 02, 12), stored as doubles [6][kMaxBodies] over
// the bodies' pose and twist fields.  Called once the rows and contacts are
// built and a barrier has passed: nothing reads those fields afterwards, and
// the rotation and inertia fields read here lie above them.  Ends with a
// barrier.
template <int NT>
__device__ inline void body_angular_minv(const Lds &L, int nb) {
    double *mi = reinterpret_cast<double *>(L.b);
    static_assert(12 <= BUF && BR >= 12 && BII >= 12, "six doubles per body below the fields still in use");
    const int b = threadIdx.x;
    if (b < nb) {
        double m[6];
        double R[9], ii[3];
        for (int k = 0; k < 9; ++k) R[k] = L.bf(BR + k, b);
        for (int k = 0; k < 3; ++k) ii[k] = L.bf(BII + k, b);
        const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
        for (int e = 0; e < 6; ++e) {
            const int i = ij[e][0], j = ij[e][1];
            double v = (R[3 * i] * ii[0]) * R[3 * j];
            v = __builtin_fma(R[3 * i + 1] * ii[1], R[3 * j + 1], v);
            m[e] = __builtin_fma(R[3 * i + 2] * ii[2], R[3 * j + 2], v);
        }
        for (int e = 0; e < 6; ++e) mi[e * kMaxBodies + b] = m[e];
    }
    __syncthreads();
}

// Row r of the product after a gather, given w_a, w_b = M^-1 g of its bodies.
// (drive rows add their regularisation: D = J M^-1 J^T + R, Eq. 4, so row r
// of D~ x gains p_r R_r p_r x_r)
__device__ inline float delassus_row_w(const Lds &L, const float *vp, int r, const double wa[6], const double wbv[6],
                                       bool has_b, float xr) {
    double a0 = 0.0, a1 = 0.0;
    for (int c = 0; c < 6; ++c) a0 += (double)L.rf(RJ + c, r) * wa[c];
    if (has_b)
        for (int c = 0; c < 6; ++c) a1 += (double)L.rf(RJ + 6 + c, r) * wbv[c];
    const double pr = (double)vp[r];
    return (float)((a0 + a1 + (double)L.rf(RREG, r) * pr * (double)xr) * pr);
}

__device__ inline float delassus_row(const Lds &L, const float *vp, int r, float xr) {
    int ia = L.ri(RIA, r), ib = L.ri(RIB, r);
    double wa[6], wbv[6];
    body_minv64(L, ia, wa);
    if (ib >= 0) body_minv64(L, ib, wbv);
    return delassus_row_w(L, vp, r, wa, wbv, ib >= 0, xr);
}

// Full product out = D~ x (gather, then every row).  Ends with a barrier.
template <int NT>
__device__ inline void delassus_apply(const Lds &L, int m, int nb, const float *vp, const float *x, float *out) {
    delassus_gather<NT>(L, nb, vp, x);
    for (int r = threadIdx.x; r < m; r += NT) out[r] = delassus_row(L, vp, r, x[r]);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the fused step kernel
// ---------------------------------------------------------------------------

// One step of world w (every phase of the step; the workgroup owns the
// world).  step is the step index that keys the actuation noise; k the
// position of the step inside the launch.
// Cholesky of D~ + diag(eta + rho) held packed in A, then the explicit
// inverse of the factor in place (Alg. 1 step 1), for a refactorization
// after the adaptive penalty changed rho: the step's own factorization
// (the same operations) is written out where the step factors first, so
// this out-of-line copy leaves that code and its schedule alone.  Returns
// nonzero when a pivot is not positive.
template <int MC, int NT>
__device__ __attribute__((noinline)) int factor_invert_again(const Lds &L, float *A, int m, int *s_int,
                                                             const StepArgs &a, int w) {
    const int tid = threadIdx.x;
    // ---- Cholesky of D~ + diag(eta + rho), in place (Alg. 1 step 1):
    //      right-looking over 16x16 tiles.  Wave 0 factors a diagonal tile in
    //      registers (lane r holds row r) and forms its inverse; the panel
    //      below is multiplied by that inverse on the matrix cores; the
    //      trailing tiles get their rank-16 update on the matrix cores.  With
    //      one step of lookahead, wave 0 updates and factors the next
    //      diagonal tile while the other waves update the rest.
    {
        const int T = (m + 15) >> 4;
        float *Xs = L.red;  // 16x16 inverse of the current diagonal factor tile (red + wb are free here)
        const int lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
        constexpr int NW = NT / 64;
        // one wave alone: at most two tile rows, so every trailing update is
        // the next diagonal tile (wave 0's); the other waves' loop never runs
        static_assert(NW > 1 || MC <= 32, "a single-wave factorization covers two tile rows");
        if (tid == 0) s_int[2] = 0;
        __syncthreads();
        // factor diagonal tile K (wave 0 only) and write its inverse to Xs
        auto factor_diag = [&](int K) {
            const int k0 = 16 * K;
            const int r = lane;
            float a[16];
            const float *Rr = A + tri_row_offset(k0 + (r & 15)) + k0;
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = (r < 16 && c <= r) ? Rr[c] : 0.f;
            bool ok = true;
            float ild[16];  // 1 / l_kk (the same in every lane)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                float d = rdlane(a[k], k);
                ok = ok && (d > 0.f) && isfinite(d);
                // hardware reciprocal square root (1 ulp); l_kk = d / sqrt(d)
                float il = __builtin_amdgcn_rsqf(d), lkk = d * il;
                ild[k] = il;
                if (r == k) a[k] = lkk;
                else if (r > k) a[k] *= il;
#pragma unroll
                for (int j = k + 1; j < 16; ++j) {
                    float ljk = rdlane(a[k], j);
                    if (r >= j) a[j] -= a[k] * ljk;
                }
            }
            // column r of the tile's inverse (forward substitution)
            float xc[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                float acc = (r == rr) ? 1.f : 0.f;
#pragma unroll
                for (int kk = 0; kk < rr; ++kk) acc -= rdlane(a[kk], rr) * xc[kk];
                xc[rr] = acc * ild[rr];
            }
            if (r < 16) {
                float *Rw = A + tri_row_offset(k0 + r) + k0;
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c <= r) Rw[c] = a[c];
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) Xs[16 * rr + r] = xc[rr];  // zero above the diagonal
            }
            if (!ok && r == 0) s_int[2] = 1;
        };
        // A_IJ -= L_IK L_JK^T for one tile pair (one wave, matrix cores)
        auto update_pair = [&](int I, int J, int k0) {
            const float *Ri = A + tri_row_offset(16 * I + fr) + k0;
            const float *Rj = A + tri_row_offset(16 * J + fr) + k0;
            mfx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) acc = mfma4(Ri[4 * ch + fk], Rj[4 * ch + fk], acc);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int rr = 4 * fk + c;
                if (I != J || fr <= rr) A[tri_row_offset(16 * I + rr) + 16 * J + fr] -= acc[c];
            }
        };
#ifdef KAMX_FACTOR_TIMING
        uint64_t fsub[4] = {0, 0, 0, 0}, fmark = a.phase_clk && tid == 0 ? wall_clock64() : 0;
#define KAMX_FMARK(k)                                   \
    if (a.phase_clk && tid == 0) {                      \
        uint64_t now_ = wall_clock64();                 \
        fsub[k] += now_ - fmark;                        \
        fmark = now_;                                   \
    }
#else
#define KAMX_FMARK(k)
#endif
        if (wv == 0) factor_diag(0);
        __syncthreads();
        KAMX_FMARK(0);
        for (int K = 0; K < T; ++K) {
            if (s_int[2]) break;
            const int k0 = 16 * K;
            const int nI = T - K - 1;
            // panel: L_IK = A_IK Xkk^T for the tiles I below the diagonal,
            // one wave per tile (each wave reads its tile before overwriting it)
            for (int Ii = wv; Ii < nI; Ii += NW) {
                const int I = K + 1 + Ii;
                mfx4 acc = {0.f, 0.f, 0.f, 0.f};
                const float *Ar = A + tri_row_offset(16 * I + fr) + k0;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) acc = mfma4(Ar[4 * ch + fk], Xs[16 * fr + 4 * ch + fk], acc);
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(16 * I + 4 * fk + c) + k0 + fr] = acc[c];
            }
            __syncthreads();
            KAMX_FMARK(1);
            if (nI == 0) break;
            // trailing update A_IJ -= L_IK L_JK^T, K < J <= I.  Pair 0 is the
            // next diagonal tile: wave 0 updates and factors it; the other
            // waves take the remaining pairs.
            const int npair = nI * (nI + 1) / 2;
            if (wv == 0) {
                update_pair(K + 1, K + 1, k0);
                factor_diag(K + 1);
            } else {
                for (int p = wv; p < npair; p += NW - 1) {
                    int Ii = (int)((sqrtf(8.f * (float)p + 1.f) - 1.f) * 0.5f);
                    while ((Ii + 1) * (Ii + 2) / 2 <= p) ++Ii;
                    while (Ii * (Ii + 1) / 2 > p) --Ii;
                    const int Jj = p - Ii * (Ii + 1) / 2;
                    update_pair(K + 1 + Ii, K + 1 + Jj, k0);
                }
            }
            __syncthreads();
            KAMX_FMARK(2);
        }
#ifdef KAMX_FACTOR_TIMING
        if (a.phase_clk && tid == 0)
            for (int q = 0; q < 3; ++q) a.phase_clk[16 * w + 8 + q] = fsub[q];
#endif
#undef KAMX_FMARK
    }
    __syncthreads();
    const int factor_fail = s_int[2];

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 4] = wall_clock64();
    // ---- explicit inverse of the factor, in place: X = L^-1 over 16x16
    //      tiles.  Diagonal tiles are inverted in registers (one wave per
    //      tile); then tile row by tile row, M_ik = X_ii L_ik (k < i) and
    //      X_ij = -sum_{k=j}^{i-1} M_ik X_kj, one wave per tile on the
    //      matrix cores, results held in registers until every wave has read
    //      the row.
    if (!factor_fail) {
        const int T = (m + 15) >> 4;
        const int lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
        constexpr int NW = NT / 64;
        static_assert(2 * NW >= MC / 16 - 1, "two off-diagonal tiles per wave must cover a tile row");
        for (int Ti = wv; Ti < T; Ti += NW) {
            const int k0 = 16 * Ti, r = lane;
            float a[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = (r < 16 && c <= r) ? A[tri_row_offset(k0 + (r & 15)) + k0 + c] : 0.f;
            float xc[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                float acc = (r == rr) ? 1.f : 0.f;
#pragma unroll
                for (int kk = 0; kk < rr; ++kk) acc -= rdlane(a[kk], rr) * xc[kk];
                xc[rr] = acc * __builtin_amdgcn_rcpf(rdlane(a[rr], rr));  // hardware reciprocal (1 ulp)
            }
            if (r < 16) {
#pragma unroll
                for (int rr = 0; rr < 16; ++rr)
                    if (rr >= r) A[tri_row_offset(k0 + rr) + k0 + r] = xc[rr];
            }
        }
        __syncthreads();
        for (int Ti = 1; Ti < T; ++Ti) {
            const int i0 = 16 * Ti;
            // M_ik = X_ii L_ik in place
            for (int Tk = wv; Tk < Ti; Tk += NW) {
                mfx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    acc = mfma4(tri_at(A, i0 + fr, i0 + 4 * ch + fk),
                                A[tri_row_offset(i0 + 4 * ch + fk) + 16 * Tk + fr], acc);
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(i0 + 4 * fk + c) + 16 * Tk + fr] = acc[c];
            }
            __syncthreads();
            // X_ij = -sum_k M_ik X_kj (two tiles per wave at most: 14 tile rows, 8 waves)
            mfx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int Tj = wv + q * NW;
                if (Tj >= Ti) continue;
                // the diagonal tile X_jj (lower triangular) first, then the full
                // tiles below it with unconditional loads, alternating between
                // two accumulators so consecutive products do not wait on
                // each other
                mfx4 acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
                const float *Mr = A + tri_row_offset(i0 + fr);
                const int jc = 16 * Tj + fr;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) {
                    const int kr = 16 * Tj + 4 * ch + fk;
                    acc = mfma4(Mr[16 * Tj + 4 * ch + fk], tri_at(A, kr, jc), acc);
                }
                for (int Tk = Tj + 1; Tk < Ti; ++Tk) {
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) {
                        const int kr = 16 * Tk + 4 * ch + fk;
                        const float mv = Mr[16 * Tk + 4 * ch + fk], xv = A[tri_row_offset(kr) + jc];
                        if (ch & 1) accb = mfma4(mv, xv, accb);
                        else acc = mfma4(mv, xv, acc);
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += accb[c];
                if (q == 0) acc0 = acc;
                else acc1 = acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int Tj = wv + q * NW;
                if (Tj >= Ti) continue;
                const mfx4 acc = q == 0 ? acc0 : acc1;
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(i0 + 4 * fk + c) + 16 * Tj + fr] = -acc[c];
            }
        }
        __syncthreads();
    }

    return factor_fail;
}

// D~ + diag(eta + rho) rebuilt into A after the adaptive penalty changed
// rho: the pairs, products and order of the step's assembly, with the
// Jacobi scales of the step and W = M^-1 J^T formed per pair from the bodies
// (the vector region that held W now holds the iterates).  Uses the
// reduction area (free between iterations) for the pair-task offsets.
template <int MC, int NT>
__device__ __attribute__((noinline)) void reassemble(const Lds &L, float *A, int m, int nb, const float *vp,
                                                     const float *vrho, float eta) {
    const int tid = threadIdx.x;
    const int Mp = (m + 15) & ~15;
    const int n4 = tri_row_offset(Mp) >> 2;
    for (int k = tid; k < n4; k += NT) reinterpret_cast<float4 *>(A)[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    int *toff = reinterpret_cast<int *>(L.red);
    if (tid == 0) {
        toff[0] = 0;
        for (int b = 0; b < nb; ++b) {
            int kb = L.inc_off[b + 1] - L.inc_off[b];
            toff[b + 1] = toff[b] + kb * (kb + 1) / 2;
        }
    }
    __syncthreads();
    if (tid >= m && tid < Mp) A[tri_row_offset(tid) + tid] = 1.f;
    auto wside = [&](int r, int sd, float out[6]) {
        const int b = L.ri(sd ? RIB : RIA, r);
        float in[6];
        for (int k = 0; k < 6; ++k) in[k] = L.rf(RJ + 6 * sd + k, r);
        if (b >= 0) apply_minv(L, b, in, out);
        else
            for (int k = 0; k < 6; ++k) out[k] = 0.f;
    };
    const int ntask = toff[nb];
    for (int t = tid; t < ntask; t += NT) {
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (toff[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        const int b = lo;
        const int loc = t - toff[b];
        int u = (int)((sqrtf(8.f * (float)loc + 1.f) - 1.f) * 0.5f);
        while ((u + 1) * (u + 2) / 2 <= loc) ++u;
        while (u * (u + 1) / 2 > loc) --u;
        const int v = loc - u * (u + 1) / 2;
        const int ri_ = L.inc_list[L.inc_off[b] + u] >> 1;
        const int rj_ = L.inc_list[L.inc_off[b] + v] >> 1;
        const int ia = L.ri(RIA, ri_), ib = L.ri(RIB, ri_), ja = L.ri(RIA, rj_), jb = L.ri(RIB, rj_);
        int first = 1 << 30;
        if (ia == ja || ia == jb) first = ia;
        if (ib >= 0 && (ib == ja || ib == jb) && ib < first) first = ib;
        if (first != b) continue;
        float acc = 0.f, wv[6];
        if (ia == ja) {
            wside(rj_, 0, wv);
            for (int k = 0; k < 6; ++k) acc += L.rf(RJ + k, ri_) * wv[k];
        }
        if (ia == jb) {
            wside(rj_, 1, wv);
            for (int k = 0; k < 6; ++k) acc += L.rf(RJ + k, ri_) * wv[k];
        }
        if (ib >= 0 && ib == ja) {
            wside(rj_, 0, wv);
            for (int k = 0; k < 6; ++k) acc += L.rf(RJ + 6 + k, ri_) * wv[k];
        }
        if (ib >= 0 && ib == jb) {
            wside(rj_, 1, wv);
            for (int k = 0; k < 6; ++k) acc += L.rf(RJ + 6 + k, ri_) * wv[k];
        }
        if (ri_ == rj_) acc += L.rf(RREG, ri_);
        acc *= vp[ri_] * vp[rj_];
        if (ri_ == rj_) acc += eta + vrho[ri_];
        A[tri_row_offset(ri_) + rj_] = acc;
    }
    __syncthreads();
}

template <int MC, int NT>
__device__ __attribute__((noinline)) void step_world(const StepArgs &a, int k, int *s_int) {
    extern __shared__ float4 smem4[];
    float *sm = reinterpret_cast<float *>(smem4);
    const int tid = threadIdx.x;
    // read per step (not hoisted out of the caller's step loop)
    const int w = a.bucket_worlds[blockIdx.x];
    const uint32_t step = *a.step_ctr + (uint32_t)k;
    const WorldInfo W = a.worlds[w];
    const SolverParams &P = a.p;

    Lds L;
    L.mc = MC;
    L.b = sm;
    L.j = L.b + body_floats();
    L.c = L.j + joint_floats();
    L.r = L.c + contact_floats();
    L.v = L.r + row_floats(MC);
    L.A = L.v + vec_floats(MC);
    L.red = L.A + tri_row_offset(MC);
    L.wb = reinterpret_cast<double *>(L.red + 64);
    L.qd = L.wb + 6 * kMaxBodies;
    L.inc_off = reinterpret_cast<int *>(L.red + 64 + bodyw_floats() + posed_floats());
    L.inc_list = L.inc_off + kMaxBodies + 1;
    float *A = L.A;

    const int nb = W.nb, nj = W.nj;

    if (a.phase_clk && tid == 0) {
        a.phase_clk[16 * w + 0] = wall_clock64();
        a.phase_clk[16 * w + 14] = __smid();  // compute unit that runs this world
        a.phase_clk[16 * w + 15] = __builtin_amdgcn_s_getreg(GETREG_IMMED(31, 0, HW_ID));  // raw hardware id
    }
    // ---- reset: a world whose reset body fell below the threshold restarts
    if (tid == 0) {
        int rs = 0;
        if (W.reset_body >= 0) {
            float z = a.q[7 * (W.b0 + W.reset_body) + 2];
            rs = z < P.reset_height;
        }
        s_int[0] = rs;
        if (rs && a.stage == 0) a.reset_count[w] += 1;
    }
    __syncthreads();
    const int reset = s_int[0];

    // ---- bodies: state, rotation, inverse mass properties
    for (int b = tid; b < nb; b += NT) {
        int gb = W.b0 + b;
        const float *qs = reset ? a.q0 : a.q;
        const float *us = reset ? a.u0 : a.u;
        float q[7], u6[6];
        for (int k = 0; k < 7; ++k) q[k] = qs[7 * gb + k];
        for (int k = 0; k < 6; ++k) u6[k] = us[6 * gb + k];
        // the configuration the rows are built at, in FP64: the pre-step pose,
        // or (Moreau-Jean) the half-step pose, whose joint geometry must not
        // carry FP32 rounding into the Baumgarte bias
        double qd[7];
        for (int k = 0; k < 7; ++k) qd[k] = q[k];
        if (P.integrator == KAMX_MOREAU_JEAN) {
            double u6d[6], qm[7];
            for (int k = 0; k < 6; ++k) u6d[k] = u6[k];
            advance_pose(qd, u6d, 0.5 * (double)P.dt, qm);
            for (int k = 0; k < 7; ++k) qd[k] = qm[k];
            for (int k = 0; k < 7; ++k) q[k] = (float)qm[k];
        }
        for (int k = 0; k < 7; ++k) L.qd[k * kMaxBodies + b] = qd[k];
        for (int k = 0; k < 7; ++k) L.bf(BQ + k, b) = q[k];
        for (int k = 0; k < 6; ++k) L.bf(BU + k, b) = u6[k];
        float R[9];
        rot_of_quat(q + 3, R);
        for (int k = 0; k < 9; ++k) L.bf(BR + k, b) = R[k];
        for (int k = 0; k < 3; ++k) L.bf(BII + k, b) = 1.f / a.inertia[3 * gb + k];
        L.bf(BIM, b) = 1.f / a.mass[gb];
    }
    __syncthreads();

    // ---- joints: coordinate, rate and actuation (generalized force along
    //      the coordinate: external + PD + noise)
    for (int j = tid; j < nj; j += NT) {
        int gj = W.j0 + j;
        int type = a.jint[4 * gj], la = a.jint[4 * gj + 1], lb = a.jint[4 * gj + 2], fl = a.jint[4 * gj + 3];
        const float *jf = a.jf + kJointFloats * gj;
        JointGeo g;
        joint_geo(L, jf, la, lb, g);
        float Ja[6], Jb[6];
        float c = (float)joint_coord(type, g, Ja, Jb);
        float rate = 0.f;
        for (int k = 0; k < 6; ++k) rate += Ja[k] * L.bf(BU + k, la);
        if (lb >= 0)
            for (int k = 0; k < 6; ++k) rate += Jb[k] * L.bf(BU + k, lb);
        float tau = a.ext_tau ? a.ext_tau[gj] : 0.f;
        float kp = jf[16], kd = jf[17], ref = jf[18];
        if (!(fl & kJointDriven) && (kp != 0.f || kd != 0.f)) tau += kp * (ref - c) - kd * rate;
        if ((fl & kJointActuated) && P.torque_sigma != 0.f)
            tau += P.torque_sigma * noise_normal(P.seed_lo, P.seed_hi, (uint32_t)w, step, (uint32_t)j);
        L.jfld(JTAU, j) = tau;
        for (int k = 0; k < 6; ++k) {
            L.jfld(JC + k, j) = Ja[k];
            L.jfld(JC + 6 + k, j) = Jb[k];
        }
        reinterpret_cast<int *>(L.j)[JA * kMaxJoints + j] = la;
        reinterpret_cast<int *>(L.j)[JB * kMaxJoints + j] = lb;
        reinterpret_cast<int *>(L.j)[JTF * kMaxJoints + j] = type | (fl << 4);
        a.tau_out[gj] = tau;
    }
    __syncthreads();

    // ---- feature pass of the learned warm start: the state the step starts
    //      from (positions relative to the reset body), the previous step's
    //      impulses by slot and the generalized forces of this step
    // feature t of this world (same layout as kamx_model_features)
    auto feature = [&](int t) -> float {
        const int rb = W.reset_body;
        const int rc0 = 5 * nj + W.nlim + W.ndrv;
        const int S = rc0 + 3 * a.n_contact_slots;
        if (t < 13 * nb) {
            const int b = t / 13, c = t - 13 * (t / 13);
            if (c < 3) return L.bf(BQ + c, b) - (rb >= 0 ? L.bf(BQ + c, rb) : 0.f);
            if (c < 7) return L.bf(BQ + c, b);
            return L.bf(BU + c - 7, b);
        }
        t -= 13 * nb;
        if (t < S) {
            float v = 0.f;
            if (!reset) {
                if (t < rc0) {
                    v = a.lambda[W.row_base + t];
                } else {
                    const int slot = (t - rc0) / 3, e = (t - rc0) - 3 * ((t - rc0) / 3);
                    const int nprev = a.ncontacts_out[w];
                    for (int q = 0; q < nprev && q < kMaxContacts; ++q)
                        if (a.keys[w * kMaxContacts + q] >= 0 && contact_slot(a.keys[w * kMaxContacts + q]) == slot) {
                            v = a.lambda[W.row_base + rc0 + 3 * q + e];
                            break;
                        }
                }
            }
            return v;
        }
        return L.jfld(JTAU, t - S);
    };
    if (a.stage == 1) {
        float *f = a.features + (long)w * a.n_feat;
        for (int t = tid; t < a.n_feat; t += NT) f[t] = feature(t);
        return;
    }

    // ---- learned warm start: the network predicts this world's impulses by
    //      slot, on the matrix cores with the batched kernels' operand layout
    //      and accumulation order (so the prediction has the same bits); the
    //      features are row 0 of the 16-row operand, the other rows zero.
    //      The triangle region of LDS is free until the Delassus assembly.
    if (P.warmstart == KAMX_WARM_LEARNED && !reset) {
        const MlpView &N = a.mlp;
        __bf16 *xh = reinterpret_cast<__bf16 *>(A);
        __bf16 *h1 = xh + N.fp;
        __bf16 *h2 = h1 + N.H;
        for (int t = tid; t < N.fp; t += NT) xh[t] = to_bf16(t < N.n_in ? (feature(t) - N.mu_in[t]) * N.s_in[t] : 0.f);
        __syncthreads();
        const int lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = (lane >> 4) * 8;
        constexpr int NW = NT / 64;
        const bf16x8 zero8 = {};
        auto layer = [&](const __bf16 *x, int K, const __bf16 *Wt, int nout_pad, auto &&epilogue) {
            for (int t = wv; t < nout_pad / 16; t += NW) {
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                const __bf16 *wrow = Wt + (long)(16 * t + fr) * K + fk;
                for (int k0 = 0; k0 < K; k0 += 32) {
                    const bf16x8 av = fr == 0 ? *reinterpret_cast<const bf16x8 *>(x + k0 + fk) : zero8;
                    const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(wrow + k0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
                }
                if (fk == 0) epilogue(16 * t + fr, acc[0]);  // row 0 of the block: lanes 0-15, component 0
            }
        };
        layer(xh, N.fp, N.w1, N.H, [&](int n, float v) { h1[n] = to_bf16(gelu(v + N.b1[n])); });
        __syncthreads();
        layer(h1, N.H, N.w2, N.H, [&](int n, float v) { h2[n] = to_bf16(gelu(v + N.b2[n])); });
        __syncthreads();
        float *ws = a.ws_slots + (long)w * N.n_out;
        layer(h2, N.H, N.w3, N.op, [&](int n, float v) {
            if (n < N.n_out) ws[n] = __builtin_fmaf(N.sd_out[n], v + N.b3[n], N.mu_out[n]);
        });
        __syncthreads();
    }

    // ---- free velocity of every body: u_f = u + dt M^-1 h
    for (int b = tid; b < nb; b += NT) {
        float m = 1.f / L.bf(BIM, b);
        float h[6];
        h[0] = m * P.gx;
        h[1] = m * P.gy;
        h[2] = m * P.gz;
        // gyroscopic -w x (I_w w), I_w w evaluated in the body frame
        float R[9], w3[3], t[3], Iw[3], gyro[3];
        body_rot(L, b, R);
        for (int k = 0; k < 3; ++k) w3[k] = L.bf(BU + 3 + k, b);
        mtv3(R, w3, t);
        for (int k = 0; k < 3; ++k) t[k] /= L.bf(BII + k, b);
        mv3(R, t, Iw);
        cross(w3, Iw, gyro);
        h[3] = -gyro[0];
        h[4] = -gyro[1];
        h[5] = -gyro[2];
        const int *ja = reinterpret_cast<const int *>(L.j) + JA * kMaxJoints;
        const int *jb = reinterpret_cast<const int *>(L.j) + JB * kMaxJoints;
        for (int j = 0; j < nj; ++j) {
            float tau = L.jfld(JTAU, j);
            if (tau == 0.f) continue;
            if (ja[j] == b)
                for (int k = 0; k < 6; ++k) h[k] += tau * L.jfld(JC + k, j);
            if (jb[j] == b)
                for (int k = 0; k < 6; ++k) h[k] += tau * L.jfld(JC + 6 + k, j);
        }
        float dv[6];
        apply_minv(L, b, h, dv);
        for (int k = 0; k < 6; ++k) L.bf(BUF + k, b) = L.bf(BU + k, b) + P.dt * dv[k];
    }

    // ---- contacts: explicit list, or probes below the margin (compacted in
    //      probe order by a wave ballot)
    int *cint = reinterpret_cast<int *>(L.c);
    constexpr bool kBoxFits = (long)sizeof(float) * (8L * (MC / 4) * (MC / 4 + 1)) >= (long)sizeof(BoxLds);
    if (kBoxFits && a.box_geom) {
        // boxes in a bin: contacts generated here from the poses the step
        // starts from, with the candidates in the LDS of the Delassus
        // triangle (free until the assembly)
        if constexpr (kBoxFits) {
            BoxLds &S = *reinterpret_cast<BoxLds *>(A);
            const int n = box_bin_generate<NT>(
                S, nb, a.box_geom + 4 * (long)W.b0, a.bin_wx, a.bin_wy, a.bin_margin, W.contact_cap,
                [&](int b, float c[3], float qt[4]) {
                    for (int e = 0; e < 3; ++e) c[e] = L.bf(BQ + e, b);
                    for (int e = 0; e < 4; ++e) qt[e] = L.bf(BQ + 3 + e, b);
                },
                [&](int c, int key, float gap, const float p[3], const float nn[3], float mu, int la, int lb) {
                    for (int e = 0; e < 3; ++e) {
                        L.cf(CP + e, c) = p[e];
                        L.cf(CN + e, c) = nn[e];
                    }
                    L.cf(CGAP, c) = gap;
                    L.cf(CMU, c) = mu;
                    cint[CA * kMaxContacts + c] = la;
                    cint[CB * kMaxContacts + c] = lb;
                    cint[CKEY * kMaxContacts + c] = key;
                });
            if (tid == 0) s_int[1] = n;
        }
    } else if (a.contacts) {
        int c0 = a.ccount ? w * kMaxContacts : a.coff[w];
        int n = a.ccount ? a.ccount[w] : a.coff[w + 1] - c0;
        if (n > W.contact_cap) n = W.contact_cap;
        if (n < 0) n = 0;
        if (tid == 0) s_int[1] = n;
        for (int c = tid; c < n; c += NT) {
            kamx_contact ct = a.contacts[c0 + c];
            int la = ct.body_a - W.b0;
            int lb = ct.body_b < 0 ? -1 : ct.body_b - W.b0;
            bool ok = la >= 0 && la < nb && lb < nb;
            for (int k = 0; k < 3; ++k) {
                L.cf(CP + k, c) = ct.point[k];
                L.cf(CN + k, c) = ct.normal[k];
            }
            L.cf(CGAP, c) = ct.gap;
            L.cf(CMU, c) = ct.mu;
            // an invalid body index turns the contact into an inert row pair
            cint[CA * kMaxContacts + c] = ok ? la : 0;
            cint[CB * kMaxContacts + c] = ok ? lb : -1;
            if (!ok) L.cf(CGAP, c) = 1e30f;
            cint[CKEY * kMaxContacts + c] = ct.key;
        }
    } else if (tid < 64) {
        int k = tid;
        bool act = false;
        float pw[3] = {0.f, 0.f, 0.f};
        int lbod = 0;
        float mu = 0.f;
        if (k < W.np) {
            int gp = W.p0 + k;
            lbod = a.pbody[gp];
            float pl[3] = {a.pf[4 * gp], a.pf[4 * gp + 1], a.pf[4 * gp + 2]};
            mu = a.pf[4 * gp + 3];
            // world point in FP64 (its height is the gap, which enters the
            // bias divided by dt), then rounded to FP32
            double qd[4], Rd[9], pld[3] = {pl[0], pl[1], pl[2]}, td[3];
            for (int e = 0; e < 4; ++e) qd[e] = L.qd[(3 + e) * kMaxBodies + lbod];
            rot_of_quat(qd, Rd);
            mv3(Rd, pld, td);
            for (int e = 0; e < 3; ++e) pw[e] = (float)(L.qd[e * kMaxBodies + lbod] + td[e]);
            act = pw[2] < P.contact_margin;
        }
        unsigned long long mask = __ballot(act);
        int slot = __popcll(mask & ((1ull << k) - 1ull));
        if (act && slot < W.contact_cap) {
            for (int e = 0; e < 3; ++e) L.cf(CP + e, slot) = pw[e];
            L.cf(CN + 0, slot) = 0.f;
            L.cf(CN + 1, slot) = 0.f;
            L.cf(CN + 2, slot) = 1.f;
            L.cf(CGAP, slot) = pw[2];
            L.cf(CMU, slot) = mu;
            cint[CA * kMaxContacts + slot] = lbod;
            cint[CB * kMaxContacts + slot] = -1;
            cint[CKEY * kMaxContacts + slot] = k;
        }
        if (k == 0) {
            int n = __popcll(mask);
            s_int[1] = n < W.contact_cap ? n : W.contact_cap;
        }
    }
    __syncthreads();
    const int nc = s_int[1];
    const int row_lim0 = 5 * nj;
    const int row_drv0 = 5 * nj + W.nlim;
    const int row_c0 = row_drv0 + W.ndrv;
    const int m = row_c0 + 3 * nc;

    // ---- constraint rows
    for (int j = tid; j < nj; j += NT) {
        int gj = W.j0 + j;
        int type = a.jint[4 * gj], la = a.jint[4 * gj + 1], lb = a.jint[4 * gj + 2], fl = a.jint[4 * gj + 3];
        const float *jf = a.jf + kJointFloats * gj;
        JointGeo g;
        joint_geo(L, jf, la, lb, g);
        joint_rows(L, type, g, la, lb, 5 * j, P);
        if (fl & kJointLimited) {
            int rank = 0;
            const int *tf = reinterpret_cast<const int *>(L.j) + JTF * kMaxJoints;
            for (int k = 0; k < j; ++k) rank += (tf[k] >> 4) & kJointLimited ? 1 : 0;
            float Ja[6], Jb[6];
            double c = joint_coord(type, g, Ja, Jb);
            double lo = jf[14], hi = jf[15];
            bool use_lo;
            if (isnan(hi)) use_lo = true;
            else if (isnan(lo)) use_lo = false;
            else use_lo = (c - lo) <= (hi - c);
            float sg = use_lo ? 1.f : -1.f;
            float gval = (float)(use_lo ? c - lo : hi - c);
            for (int k = 0; k < 6; ++k) {
                Ja[k] *= sg;
                Jb[k] *= sg;
            }
            put_row(L, row_lim0 + rank, Ja, la, Jb, lb, gval, kRowLimit, 0.f, P);
        }
        if (fl & kJointDriven) {
            // drive row (Sec. 3 implicit PD, armature, damping; Eq. 2 R, v*):
            // along the coordinate c the impulse over the step is
            // dt [kp (ref - c - h c'+) - (kd + d) c'+ - I_a (c'+ - c'-) / dt],
            // i.e. J_c u+ + R lambda + v* = 0 with K = kp h + kd + d + I_a / dt,
            // R = 1 / (dt K), v* = -(kp (ref - c) + I_a c'- / dt) / K
            int rank = 0;
            const int *tf = reinterpret_cast<const int *>(L.j) + JTF * kMaxJoints;
            for (int k = 0; k < j; ++k) rank += (tf[k] >> 4) & kJointDriven ? 1 : 0;
            float Ja[6], Jb[6];
            const double c = joint_coord(type, g, Ja, Jb);
            float rate = 0.f;
            for (int k = 0; k < 6; ++k) rate += Ja[k] * L.bf(BU + k, la);
            if (lb >= 0)
                for (int k = 0; k < 6; ++k) rate += Jb[k] * L.bf(BU + k, lb);
            const float h = P.integrator == KAMX_MOREAU_JEAN ? 0.5f * P.dt : P.dt;
            const float kp = jf[16], kd = jf[17], ref = jf[18], damp = jf[19], arm = jf[20];
            const float K = kp * h + kd + damp + arm / P.dt;
            const int r = row_drv0 + rank;
            put_row(L, r, Ja, la, Jb, lb, 0.f, kRowBilateral, 0.f, P);
            L.rf(RBIAS, r) = -(float)((double)kp * ((double)ref - c) + (double)arm * (double)rate / (double)P.dt) / K;
            L.rf(RREG, r) = 1.f / (P.dt * K);
        }
    }
    for (int c = tid; c < nc; c += NT) {
        float p[3], n[3], t1[3], t2[3];
        for (int k = 0; k < 3; ++k) {
            p[k] = L.cf(CP + k, c);
            n[k] = L.cf(CN + k, c);
        }
        tangents(n, t1, t2);
        const float *dirs[3] = {n, t1, t2};
        int la = cint[CA * kMaxContacts + c], lb = cint[CB * kMaxContacts + c];
        float arm_a[3], arm_b[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < 3; ++k) {
            arm_a[k] = p[k] - L.bf(BQ + k, la);
            if (lb >= 0) arm_b[k] = p[k] - L.bf(BQ + k, lb);
        }
        for (int e = 0; e < 3; ++e) {
            float Ja[6], Jb[6], cc[3];
            cross(arm_a, dirs[e], cc);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = dirs[e][k];
                Ja[3 + k] = cc[k];
            }
            cross(arm_b, dirs[e], cc);
            for (int k = 0; k < 3; ++k) {
                Jb[k] = -dirs[e][k];
                Jb[3 + k] = -cc[k];
            }
            put_row(L, row_c0 + 3 * c + e, Ja, la, Jb, lb, e == 0 ? L.cf(CGAP, c) : 0.f,
                    e == 0 ? kRowNormal : kRowTangent, L.cf(CMU, c), P);
        }
    }
    __syncthreads();

    // ---- body -> row incidence lists (CSR, rows in increasing order), one
    //      wave per body at a time, compacted with ballots
    {
        constexpr int NWAVE = NT / 64;
        const int lane = tid & 63, wave = tid >> 6;
        for (int b = wave; b < nb; b += NWAVE) {
            int cnt = 0;
            for (int r0 = 0; r0 < m; r0 += 64) {
                int r = r0 + lane;
                bool f = r < m && (L.ri(RIA, r) == b || L.ri(RIB, r) == b);
                cnt += __popcll(__ballot(f));
            }
            if (lane == 0) L.inc_off[b + 1] = cnt;
        }
        __syncthreads();
        if (tid == 0) {
            L.inc_off[0] = 0;
            for (int b = 0; b < nb; ++b) L.inc_off[b + 1] += L.inc_off[b];
        }
        __syncthreads();
        for (int b = wave; b < nb; b += NWAVE) {
            int base = L.inc_off[b];
            for (int r0 = 0; r0 < m; r0 += 64) {
                int r = r0 + lane;
                int side = -1;
                if (r < m) {
                    if (L.ri(RIA, r) == b) side = 0;
                    else if (L.ri(RIB, r) == b) side = 1;
                }
                unsigned long long msk = __ballot(side >= 0);
                if (side >= 0) L.inc_list[base + __popcll(msk & ((1ull << lane) - 1ull))] = (r << 1) | side;
                base += __popcll(msk);
            }
        }
        __syncthreads();
    }
    static_assert(kMaxBodies <= NT, "one thread per body");
    body_angular_minv<NT>(L, nb);

    // ---- W = M^-1 J^T for both sides of every row (in the vector region)
    float *Wv = L.v;  // [12][MC]
    for (int r = tid; r < m; r += NT) {
        for (int s = 0; s < 2; ++s) {
            int b = L.ri(s ? RIB : RIA, r);
            float in[6], out[6];
            for (int k = 0; k < 6; ++k) in[k] = L.rf(RJ + 6 * s + k, r);
            if (b >= 0) apply_minv(L, b, in, out);
            else
                for (int k = 0; k < 6; ++k) out[k] = 0.f;
            for (int k = 0; k < 6; ++k) Wv[(6 * s + k) * MC + r] = out[k];
        }
    }
    __syncthreads();

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 1] = wall_clock64();
    // ---- Jacobi scales (Sec. 4.1) from the diagonal D_ii = J_i . W_i: per
    //      row for bilateral and limit rows, one scalar per contact block
    const int i = tid;
    float *vp = L.vec(VP), *vrho = L.vec(VRHO), *vvt = L.vec(VVT);
    float *tdiag = L.vec(VCOL), *tp = L.vec(VAUX);  // free fields above W
    const int kind_row = i < m ? L.ri(RKIND, i) : -1;
    if (i < m) {
        float dsum = L.rf(RREG, i);  // D_ii = J_i M^-1 J_i^T + R_ii
        for (int k = 0; k < 12; ++k) dsum += L.rf(RJ + k, i) * Wv[k * MC + i];
        tdiag[i] = dsum;
    }
    __syncthreads();
    if (i < m) {
        if (kind_row == kRowNormal) {
            float t = (tdiag[i] + tdiag[i + 1] + tdiag[i + 2]) * (1.f / 3.f);
            float sc = (P.precond && t > 0.f) ? 1.f / sqrtf(t) : 1.f;
            tp[i] = tp[i + 1] = tp[i + 2] = sc;
        } else if (kind_row != kRowTangent) {
            float t = tdiag[i];
            tp[i] = (P.precond && t > 0.f) ? 1.f / sqrtf(t) : 1.f;
        }
    }
    __syncthreads();
    const float pi_reg = i < m ? tp[i] : 1.f;

    // ---- D~ = P J M^-1 J^T P + diag(eta + rho), packed lower triangle (rows
    //      padded to 4 floats).  Zero-fill, then every nonzero pair (i >= j)
    //      is formed once, by the first body the two rows share: the pairs of
    //      each body's incidence list are spread evenly over the threads.
    {
        const int Mp = (m + 15) & ~15;
        const int n4 = tri_row_offset(Mp) >> 2;
        for (int k = tid; k < n4; k += NT) reinterpret_cast<float4 *>(A)[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        int *toff = reinterpret_cast<int *>(L.red);  // [nb + 1] pair-task offsets (red/wb free here)
        if (tid == 0) {
            toff[0] = 0;
            for (int b = 0; b < nb; ++b) {
                int kb = L.inc_off[b + 1] - L.inc_off[b];
                toff[b + 1] = toff[b] + kb * (kb + 1) / 2;
            }
        }
        __syncthreads();
        if (i >= m && i < Mp) A[tri_row_offset(i) + i] = 1.f;  // identity rows up to a multiple of 16
        const int ntask = toff[nb];
        for (int t = tid; t < ntask; t += NT) {
            int lo = 0, hi = nb - 1;  // body b with toff[b] <= t < toff[b+1]
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (toff[mid] <= t) lo = mid;
                else hi = mid - 1;
            }
            const int b = lo;
            const int loc = t - toff[b];
            int u = (int)((sqrtf(8.f * (float)loc + 1.f) - 1.f) * 0.5f);
            while ((u + 1) * (u + 2) / 2 <= loc) ++u;
            while (u * (u + 1) / 2 > loc) --u;
            const int v = loc - u * (u + 1) / 2;
            const int ri_ = L.inc_list[L.inc_off[b] + u] >> 1;
            const int rj_ = L.inc_list[L.inc_off[b] + v] >> 1;
            const int ia = L.ri(RIA, ri_), ib = L.ri(RIB, ri_), ja = L.ri(RIA, rj_), jb = L.ri(RIB, rj_);
            int first = 1 << 30;
            if (ia == ja || ia == jb) first = ia;
            if (ib >= 0 && (ib == ja || ib == jb) && ib < first) first = ib;
            if (first != b) continue;
            float acc = 0.f;
            if (ia == ja)
                for (int k = 0; k < 6; ++k) acc += L.rf(RJ + k, ri_) * Wv[k * MC + rj_];
            if (ia == jb)
                for (int k = 0; k < 6; ++k) acc += L.rf(RJ + k, ri_) * Wv[(6 + k) * MC + rj_];
            if (ib >= 0 && ib == ja)
                for (int k = 0; k < 6; ++k) acc += L.rf(RJ + 6 + k, ri_) * Wv[k * MC + rj_];
            if (ib >= 0 && ib == jb)
                for (int k = 0; k < 6; ++k) acc += L.rf(RJ + 6 + k, ri_) * Wv[(6 + k) * MC + rj_];
            if (ri_ == rj_) acc += L.rf(RREG, ri_);  // drive rows: D = J M^-1 J^T + R
            acc *= tp[ri_] * tp[rj_];
            if (ri_ == rj_) {
                const int kd = L.ri(RKIND, ri_);
                acc += P.eta + (kd == kRowBilateral ? P.rho_bil : P.rho_c);
            }
            A[tri_row_offset(ri_) + rj_] = acc;
        }
        __syncthreads();
    }
    // the vector region held W and the scales until now: clear it (pads must
    // read as 0), then store P, rho and v~_f = P (J u_f + v*)
    for (int k = tid; k < vec_floats(MC); k += NT) L.v[k] = 0.f;
    __syncthreads();
    if (i < m) {
        vp[i] = pi_reg;
        vrho[i] = kind_row == kRowBilateral ? P.rho_bil : P.rho_c;
        float v = L.rf(RBIAS, i);
        int ia = L.ri(RIA, i), ib = L.ri(RIB, i);
        for (int k = 0; k < 6; ++k) v += L.rf(RJ + k, i) * L.bf(BUF + k, ia);
        if (ib >= 0)
            for (int k = 0; k < 6; ++k) v += L.rf(RJ + 6 + k, i) * L.bf(BUF + k, ib);
        vvt[i] = pi_reg * v;
    }
    __syncthreads();

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 2] = wall_clock64();
    // ---- warm start (Alg. 1 step 2; Sec. 4.1): y = x = Pi_K(lambda_ws / p),
    //      z = v~(y) + Gamma(v~(y)) on unilateral rows, 0 on bilateral rows
    float *vx = L.vec(VX), *vyh = L.vec(VYH), *vzh = L.vec(VZH), *vyp = L.vec(VYP), *vzp = L.vec(VZP);
    float *vrhs = L.vec(VRHS), *vt = L.vec(VT), *vxn = L.vec(VXN), *vws = L.vec(VWS), *vaux = L.vec(VAUX);
    float *vrinv = L.vec(VCOL), *vdx = L.vec(VDX);  // vrinv: 1/rho per row inside the iteration loop
    const int wmode = reset ? KAMX_WARM_COLD : P.warmstart;
    const int kind_i = i < m ? L.ri(RKIND, i) : -1;
    const bool owner = i < m && kind_i != kRowTangent;
    const int blk = kind_i == kRowNormal ? 3 : 1;
    if (wmode != KAMX_WARM_COLD) {
        if (i < m) {
            float lw = 0.f;
            if (wmode == KAMX_WARM_EXTERNAL) {
                lw = a.lambda_ext[W.row_base + i];
            } else if (wmode == KAMX_WARM_LEARNED) {
                // network output by slot: joint, limit and drive rows in
                // order, then three slots per contact slot (contact_slot)
                const float *ws = a.ws_slots + (long)w * a.mlp.n_out;
                if (i < row_c0) {
                    lw = ws[i];
                } else {
                    int c = (i - row_c0) / 3, e = (i - row_c0) % 3;
                    int key = cint[CKEY * kMaxContacts + c];
                    int sl = key >= 0 ? contact_slot(key) : -1;
                    lw = sl >= 0 && sl < a.n_contact_slots ? ws[row_c0 + 3 * sl + e] : 0.f;
                }
            } else if (i < row_c0) {
                lw = a.lambda[W.row_base + i];
            } else {
                // previous-step cache matched by contact key
                int c = (i - row_c0) / 3, e = (i - row_c0) % 3;
                int key = cint[CKEY * kMaxContacts + c];
                int nprev = a.ncontacts_out[w];
                for (int k = 0; k < nprev && k < kMaxContacts; ++k)
                    if (a.keys[w * kMaxContacts + k] == key) {
                        lw = a.lambda[W.row_base + row_c0 + 3 * k + e];
                        break;
                    }
            }
            vws[i] = isfinite(lw) ? lw / vp[i] : 0.f;
        }
        __syncthreads();
        if (owner) {
            if (kind_i == kRowNormal) {
                float o0, o1, o2;
                proj_cone(L.rf(RMU, i), vws[i], vws[i + 1], vws[i + 2], o0, o1, o2);
                vyp[i] = o0;
                vyp[i + 1] = o1;
                vyp[i + 2] = o2;
            } else if (kind_i == kRowLimit) {
                vyp[i] = fmaxf(vws[i], 0.f);
            } else {
                vyp[i] = vws[i];
            }
        }
        __syncthreads();
        delassus_apply<NT>(L, m, nb, vp, vyp, vdx);  // D~ y0 (x0 = y0)
        if (owner) {
            float v0 = vdx[i] + vvt[i];
            if (kind_i == kRowNormal) {
                float v1 = vdx[i + 1] + vvt[i + 1], v2 = vdx[i + 2] + vvt[i + 2];
                vzp[i] = v0 + L.rf(RMU, i) * sqrtf(v1 * v1 + v2 * v2);
                vzp[i + 1] = v1;
                vzp[i + 2] = v2;
            } else if (kind_i == kRowLimit) {
                vzp[i] = v0;
            } else {
                vzp[i] = 0.f;
            }
            _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk) {
                vx[i + e] = vyp[i + e];
                vyh[i + e] = vyp[i + e];
                vzh[i + e] = vzp[i + e];
            }
        }
        __syncthreads();
    }

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 3] = wall_clock64();
    // ---- Cholesky of D~ + diag(eta + rho), in place (Alg. 1 step 1):
    //      right-looking over 16x16 tiles.  Wave 0 factors a diagonal tile in
    //      registers (lane r holds row r) and forms its inverse; the panel
    //      below is multiplied by that inverse on the matrix cores; the
    //      trailing tiles get their rank-16 update on the matrix cores.  With
    //      one step of lookahead, wave 0 updates and factors the next
    //      diagonal tile while the other waves update the rest.
    {
        const int T = (m + 15) >> 4;
        float *Xs = L.red;  // 16x16 inverse of the current diagonal factor tile (red + wb are free here)
        const int lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
        constexpr int NW = NT / 64;
        // one wave alone: at most two tile rows, so every trailing update is
        // the next diagonal tile (wave 0's); the other waves' loop never runs
        static_assert(NW > 1 || MC <= 32, "a single-wave factorization covers two tile rows");
        if (tid == 0) s_int[2] = 0;
        __syncthreads();
        // factor diagonal tile K (wave 0 only) and write its inverse to Xs
        auto factor_diag = [&](int K) {
            const int k0 = 16 * K;
            const int r = lane;
            float a[16];
            const float *Rr = A + tri_row_offset(k0 + (r & 15)) + k0;
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = (r < 16 && c <= r) ? Rr[c] : 0.f;
            bool ok = true;
            float ild[16];  // 1 / l_kk (the same in every lane)
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                float d = rdlane(a[k], k);
                ok = ok && (d > 0.f) && isfinite(d);
                // hardware reciprocal square root (1 ulp); l_kk = d / sqrt(d)
                float il = __builtin_amdgcn_rsqf(d), lkk = d * il;
                ild[k] = il;
                if (r == k) a[k] = lkk;
                else if (r > k) a[k] *= il;
#pragma unroll
                for (int j = k + 1; j < 16; ++j) {
                    float ljk = rdlane(a[k], j);
                    if (r >= j) a[j] -= a[k] * ljk;
                }
            }
            // column r of the tile's inverse (forward substitution)
            float xc[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                float acc = (r == rr) ? 1.f : 0.f;
#pragma unroll
                for (int kk = 0; kk < rr; ++kk) acc -= rdlane(a[kk], rr) * xc[kk];
                xc[rr] = acc * ild[rr];
            }
            if (r < 16) {
                float *Rw = A + tri_row_offset(k0 + r) + k0;
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c <= r) Rw[c] = a[c];
#pragma unroll
                for (int rr = 0; rr < 16; ++rr) Xs[16 * rr + r] = xc[rr];  // zero above the diagonal
            }
            if (!ok && r == 0) s_int[2] = 1;
        };
        // A_IJ -= L_IK L_JK^T for one tile pair (one wave, matrix cores)
        auto update_pair = [&](int I, int J, int k0) {
            const float *Ri = A + tri_row_offset(16 * I + fr) + k0;
            const float *Rj = A + tri_row_offset(16 * J + fr) + k0;
            mfx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) acc = mfma4(Ri[4 * ch + fk], Rj[4 * ch + fk], acc);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int rr = 4 * fk + c;
                if (I != J || fr <= rr) A[tri_row_offset(16 * I + rr) + 16 * J + fr] -= acc[c];
            }
        };
#ifdef KAMX_FACTOR_TIMING
        uint64_t fsub[4] = {0, 0, 0, 0}, fmark = a.phase_clk && tid == 0 ? wall_clock64() : 0;
#define KAMX_FMARK(k)                                   \
    if (a.phase_clk && tid == 0) {                      \
        uint64_t now_ = wall_clock64();                 \
        fsub[k] += now_ - fmark;                        \
        fmark = now_;                                   \
    }
#else
#define KAMX_FMARK(k)
#endif
        if (wv == 0) factor_diag(0);
        __syncthreads();
        KAMX_FMARK(0);
        for (int K = 0; K < T; ++K) {
            if (s_int[2]) break;
            const int k0 = 16 * K;
            const int nI = T - K - 1;
            // panel: L_IK = A_IK Xkk^T for the tiles I below the diagonal,
            // one wave per tile (each wave reads its tile before overwriting it)
            for (int Ii = wv; Ii < nI; Ii += NW) {
                const int I = K + 1 + Ii;
                mfx4 acc = {0.f, 0.f, 0.f, 0.f};
                const float *Ar = A + tri_row_offset(16 * I + fr) + k0;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) acc = mfma4(Ar[4 * ch + fk], Xs[16 * fr + 4 * ch + fk], acc);
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(16 * I + 4 * fk + c) + k0 + fr] = acc[c];
            }
            __syncthreads();
            KAMX_FMARK(1);
            if (nI == 0) break;
            // trailing update A_IJ -= L_IK L_JK^T, K < J <= I.  Pair 0 is the
            // next diagonal tile: wave 0 updates and factors it; the other
            // waves take the remaining pairs.
            const int npair = nI * (nI + 1) / 2;
            if (wv == 0) {
                update_pair(K + 1, K + 1, k0);
                factor_diag(K + 1);
            } else {
                for (int p = wv; p < npair; p += NW - 1) {
                    int Ii = (int)((sqrtf(8.f * (float)p + 1.f) - 1.f) * 0.5f);
                    while ((Ii + 1) * (Ii + 2) / 2 <= p) ++Ii;
                    while (Ii * (Ii + 1) / 2 > p) --Ii;
                    const int Jj = p - Ii * (Ii + 1) / 2;
                    update_pair(K + 1 + Ii, K + 1 + Jj, k0);
                }
            }
            __syncthreads();
            KAMX_FMARK(2);
        }
#ifdef KAMX_FACTOR_TIMING
        if (a.phase_clk && tid == 0)
            for (int q = 0; q < 3; ++q) a.phase_clk[16 * w + 8 + q] = fsub[q];
#endif
#undef KAMX_FMARK
    }
    __syncthreads();
    const int factor_fail = s_int[2];

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 4] = wall_clock64();
    // ---- explicit inverse of the factor, in place: X = L^-1 over 16x16
    //      tiles.  Diagonal tiles are inverted in registers (one wave per
    //      tile); then tile row by tile row, M_ik = X_ii L_ik (k < i) and
    //      X_ij = -sum_{k=j}^{i-1} M_ik X_kj, one wave per tile on the
    //      matrix cores, results held in registers until every wave has read
    //      the row.
    if (!factor_fail) {
        const int T = (m + 15) >> 4;
        const int lane = tid & 63, wv = tid >> 6, fr = lane & 15, fk = lane >> 4;
        constexpr int NW = NT / 64;
        static_assert(2 * NW >= MC / 16 - 1, "two off-diagonal tiles per wave must cover a tile row");
        for (int Ti = wv; Ti < T; Ti += NW) {
            const int k0 = 16 * Ti, r = lane;
            float a[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) a[c] = (r < 16 && c <= r) ? A[tri_row_offset(k0 + (r & 15)) + k0 + c] : 0.f;
            float xc[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                float acc = (r == rr) ? 1.f : 0.f;
#pragma unroll
                for (int kk = 0; kk < rr; ++kk) acc -= rdlane(a[kk], rr) * xc[kk];
                xc[rr] = acc * __builtin_amdgcn_rcpf(rdlane(a[rr], rr));  // hardware reciprocal (1 ulp)
            }
            if (r < 16) {
#pragma unroll
                for (int rr = 0; rr < 16; ++rr)
                    if (rr >= r) A[tri_row_offset(k0 + rr) + k0 + r] = xc[rr];
            }
        }
        __syncthreads();
        for (int Ti = 1; Ti < T; ++Ti) {
            const int i0 = 16 * Ti;
            // M_ik = X_ii L_ik in place
            for (int Tk = wv; Tk < Ti; Tk += NW) {
                mfx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ch = 0; ch < 4; ++ch)
                    acc = mfma4(tri_at(A, i0 + fr, i0 + 4 * ch + fk),
                                A[tri_row_offset(i0 + 4 * ch + fk) + 16 * Tk + fr], acc);
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(i0 + 4 * fk + c) + 16 * Tk + fr] = acc[c];
            }
            __syncthreads();
            // X_ij = -sum_k M_ik X_kj (two tiles per wave at most: 14 tile rows, 8 waves)
            mfx4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int Tj = wv + q * NW;
                if (Tj >= Ti) continue;
                // the diagonal tile X_jj (lower triangular) first, then the full
                // tiles below it with unconditional loads, alternating between
                // two accumulators so consecutive products do not wait on
                // each other
                mfx4 acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
                const float *Mr = A + tri_row_offset(i0 + fr);
                const int jc = 16 * Tj + fr;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) {
                    const int kr = 16 * Tj + 4 * ch + fk;
                    acc = mfma4(Mr[16 * Tj + 4 * ch + fk], tri_at(A, kr, jc), acc);
                }
                for (int Tk = Tj + 1; Tk < Ti; ++Tk) {
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) {
                        const int kr = 16 * Tk + 4 * ch + fk;
                        const float mv = Mr[16 * Tk + 4 * ch + fk], xv = A[tri_row_offset(kr) + jc];
                        if (ch & 1) accb = mfma4(mv, xv, accb);
                        else acc = mfma4(mv, xv, acc);
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] += accb[c];
                if (q == 0) acc0 = acc;
                else acc1 = acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int Tj = wv + q * NW;
                if (Tj >= Ti) continue;
                const mfx4 acc = q == 0 ? acc0 : acc1;
#pragma unroll
                for (int c = 0; c < 4; ++c) A[tri_row_offset(i0 + 4 * fk + c) + 16 * Tj + fr] = -acc[c];
            }
        }
        __syncthreads();
    }

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 5] = wall_clock64();
    // ---- PADMM (Alg. 1 steps 3-10).  The x-update of step 5 is computed as
    //      x + X^T X (rhs - (D~ + eta + rho) x): one refinement step from the
    //      previous iterate with the FP32 factor inverse and an FP64
    //      matrix-free residual, so the fixed point solves the linear system
    //      to the accuracy of the residual, not to cond(D~) times FP32 epsilon.
    const float eta = P.eta;
    const float mu_i = i < m ? L.rf(RMU, i) : 0.f;
    // Inside the iteration loop row io = tid / 2 belongs to the lane pair
    // (2 io, 2 io + 1): the pair evaluates the row's matrix-free product
    // (even lane body a's side, odd lane body b's), and the even lane of a
    // block's first row owns the block, so owner work spreads over every
    // wave and a contact's three rows go to three pairs.
    const int io = tid >> 1, hh = tid & 1;
    const int kind_o = io < m ? L.ri(RKIND, io) : -1;
    const bool owner_o = io < m && kind_o != kRowTangent && hh == 0;
    const int blk_o = kind_o == kRowNormal ? 3 : 1;
    float rho_o = io < m ? vrho[io] : 1.f;  // changes only with the adaptive penalty
    const float mu_o = io < m ? L.rf(RMU, io) : 0.f;
    float a_k = 1.f, c_prev = INFINITY;
    int it = 0, status = 0;
    float rp = 0.f, rd = 0.f, rc = 0.f, rncp = 0.f;
    const int N = P.fixed_iters > 0 ? P.fixed_iters : P.max_iters;
    const int n_uni = W.nlim + 3 * nc;  // limit and contact rows: what the adaptive penalty acts on
    if (i < m) vrinv[i] = 1.f / vrho[i];  // rho is fixed for the solve: divide once
    if (factor_fail) {
        status = KAMX_WORLD_FACTOR_FAIL;
        rp = rd = rc = rncp = NAN;
        if (i < m) vyp[i] = 0.f;
    } else {
        if (wmode == KAMX_WARM_COLD && i < m) {
            vx[i] = vyh[i] = vzh[i] = vyp[i] = vzp[i] = vdx[i] = 0.f;
        }
        bool converged = false;
        float s_own = 0.f;
        // gather balance for the loop: bodies with more than half the longest
        // incidence list go first and take four threads per component, as
        // far as 12 (nb + nh) <= T allows for the bucket's default workgroup
        // size T (the same bodies, so the same sums, at every size: a
        // four-thread body adds its rows in another order than a two-thread
        // one); the order is bytes in the aux
        // field (free inside the loop). Wave 0 builds it, lane b for body b
        // (nb <= 64): a wave max, then ranks from ballots.
        static_assert(kMaxBodies <= 64 && kMaxBodies + 1 <= 4 * MC, "gather order: one lane per body, bytes in aux");
        unsigned char *gorder = reinterpret_cast<unsigned char *>(vaux);
        if (tid < 64) {
            const int kb = tid < nb ? L.inc_off[tid + 1] - L.inc_off[tid] : 0;
            int kmax = kb;
            for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o));
            const unsigned long long below = (1ull << tid) - 1ull;
            const unsigned long long hv = __ballot(tid < nb && 2 * kb > kmax);
            constexpr int kGatherThreads = default_bucket_threads(MC);
            static_assert(kGatherThreads >= 64, "gather cap from the bucket's default size");
            const int cap = max(kGatherThreads / 12 - nb, 0);
            const bool heavy = ((hv >> tid) & 1ull) && __popcll(hv & below) < cap;
            const unsigned long long hm = __ballot(heavy);
            const int nh = __popcll(hm);
            if (tid < nb)
                gorder[1 + (heavy ? __popcll(hm & below) : nh + tid - __popcll(hm & below))] = (unsigned char)tid;
            if (tid == 0) gorder[0] = (unsigned char)nh;
        }
        __syncthreads();
        const int gnh = gorder[0];
        uint64_t sub[6] = {0, 0, 0, 0, 0, 0}, tmark = 0;
        const bool timing = a.phase_clk && tid == 0;
#define KAMX_MARK(k)                                  \
    if (timing) {                                     \
        uint64_t now_ = wall_clock64();               \
        if ((k) > 0) sub[(k) > 0 ? (k) - 1 : 0] += now_ - tmark; \
        tmark = now_;                                 \
    }
        // steps 4-5: rhs = -v~_f - Gamma(z^) + eta x + rho y^ + z^, and its
        // residual against the current x (rows of this thread's block; the
        // owner computes it for the next iteration at the end of the update)
        auto own_rhs = [&]() {
            if (owner_o) {
                s_own = kind_o == kRowNormal ? mu_o * hw_sqrt(vzh[io + 1] * vzh[io + 1] + vzh[io + 2] * vzh[io + 2]) : 0.f;
                _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                    float rr = e == 0 ? rho_o : vrho[io + e];
                    float xe = vx[io + e];
                    float rhs = -vvt[io + e] - (e == 0 ? s_own : 0.f) + eta * xe + rr * vyh[io + e] + vzh[io + e];
                    vrhs[io + e] = rhs - (vdx[io + e] + (eta + rr) * xe);
                }
            }
        };
        own_rhs();
        // the solve runs in passes: a pass ends when the solve exits or when
        // the adaptive penalty changes rho, whose refactorization then runs
        // outside the iteration loop (so the loop itself carries no calls)
        int adapt_pending = 0;
        it = 1;
        for (;;) {
            for (; it <= N; ++it) {
                KAMX_MARK(0);
                __syncthreads();
                KAMX_MARK(1);
                // t = X r over groups of 4 rows: groups g and Q-1-g form a pair
                // (balanced: together they span Q+1 column quads); 16 threads per
                // pair take every 16th column quad, reading the quad of r once
                // for the 4 rows of a group. The rows of a group lie back to back,
                // 4(G+1) floats apart; the pads of the diagonal quad hold 0 and r
                // is 0 past row m, and rows past m (up to the next multiple of 16)
                // hold finite values whose sums are not stored. The eight sums
                // are reduce-scattered over the 16 lanes as in the x update.
                {
                    const int Q = (m + 3) >> 2;
                    const int g = tid >> 4, kq = tid & 15;
                    const int g1 = g, g2 = Q - 1 - g;
                    float4 s1 = make_float4(0.f, 0.f, 0.f, 0.f), s2 = s1;
                    if (g1 <= g2) {
#pragma unroll
                        for (int part = 0; part < 2; ++part) {
                            if (part == 1 && g2 == g1) break;
                            const int G = part == 0 ? g1 : g2;
                            const float *R = A + tri_row_offset(4 * G);
                            const int rl = 4 * (G + 1);
                            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
                            for (int c = kq; c <= G; c += 16) {
                                const float4 rv = *reinterpret_cast<const float4 *>(vrhs + 4 * c);
                                const float4 x0 = *reinterpret_cast<const float4 *>(R + 4 * c);
                                const float4 x1 = *reinterpret_cast<const float4 *>(R + rl + 4 * c);
                                const float4 x2 = *reinterpret_cast<const float4 *>(R + 2 * rl + 4 * c);
                                const float4 x3 = *reinterpret_cast<const float4 *>(R + 3 * rl + 4 * c);
                                acc.x += x0.x * rv.x;
                                acc.y += x1.x * rv.x;
                                acc.z += x2.x * rv.x;
                                acc.w += x3.x * rv.x;
                                acc.x += x0.y * rv.y;
                                acc.y += x1.y * rv.y;
                                acc.z += x2.y * rv.y;
                                acc.w += x3.y * rv.y;
                                acc.x += x0.z * rv.z;
                                acc.y += x1.z * rv.z;
                                acc.z += x2.z * rv.z;
                                acc.w += x3.z * rv.z;
                                acc.x += x0.w * rv.w;
                                acc.y += x1.w * rv.w;
                                acc.z += x2.w * rv.w;
                                acc.w += x3.w * rv.w;
                            }
                            if (part == 0) s1 = acc;
                            else s2 = acc;
                        }
                    }
                    const bool b3 = kq & 8, b2 = kq & 4, b1 = kq & 2;
                    const float v8[8] = {s1.x, s1.y, s1.z, s1.w, s2.x, s2.y, s2.z, s2.w};
                    float u4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        u4[k] = (b3 ? v8[k + 4] : v8[k]) + dpp<kDppMirror16>(b3 ? v8[k] : v8[k + 4]);
                    float u2[2];
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        u2[k] = (b2 ? u4[k + 2] : u4[k]) + dpp<kDppMirror8>(b2 ? u4[k] : u4[k + 2]);
                    float z = (b1 ? u2[1] : u2[0]) + dpp<kDppXor2>(b1 ? u2[0] : u2[1]);
                    z += dpp<kDppXor1>(z);
                    if (!(kq & 1) && g1 <= g2) {
                        const int i = 4 * (b3 ? g2 : g1) + (b2 ? 2 : 0) + (b1 ? 1 : 0);
                        if (i < m && (!b3 || g2 > g1)) vt[i] = z;
                    }
                }
                __syncthreads();
                KAMX_MARK(2);
                // x_new = x + X^T t over column quads: quads c and Q-1-c form a
                // pair (balanced: together they span m + 4 rows); 16 threads per
                // pair take every 16th group of 4 rows, each reading a group's t
                // and the 4 rows' entries of the quad as float4s; butterfly sum
                // over the 16 threads
                {
                    const int Q = (m + 3) >> 2;
                    const int g = tid >> 4, kq = tid & 15;
                    const int c1 = g, c2 = Q - 1 - g;
                    float4 s1 = make_float4(0.f, 0.f, 0.f, 0.f), s2 = s1;
                    if (c1 <= c2) {
#pragma unroll
                        for (int part = 0; part < 2; ++part) {
                            if (part == 1 && c2 == c1) break;
                            const int c = part == 0 ? c1 : c2;
                            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f), acc2 = acc;
                            // four consecutive rows per step (one float4 of t), every
                            // 64th row group; packed rows are padded to 4 floats and
                            // the pads hold 0, so the quad that contains the diagonal
                            // reads as-is, and t is 0 past row m (the rows there, up
                            // to the next multiple of 4, hold finite values)
                            for (int r = 4 * c + 4 * kq; r < m; r += 64) {
                                const float4 tv = *reinterpret_cast<const float4 *>(vt + r);
                                const float4 x0 = *reinterpret_cast<const float4 *>(A + tri_row_offset(r) + 4 * c);
                                const float4 x1 = *reinterpret_cast<const float4 *>(A + tri_row_offset(r + 1) + 4 * c);
                                const float4 x2 = *reinterpret_cast<const float4 *>(A + tri_row_offset(r + 2) + 4 * c);
                                const float4 x3 = *reinterpret_cast<const float4 *>(A + tri_row_offset(r + 3) + 4 * c);
                                acc.x += x0.x * tv.x;
                                acc.y += x0.y * tv.x;
                                acc.z += x0.z * tv.x;
                                acc.w += x0.w * tv.x;
                                acc2.x += x1.x * tv.y;
                                acc2.y += x1.y * tv.y;
                                acc2.z += x1.z * tv.y;
                                acc2.w += x1.w * tv.y;
                                acc.x += x2.x * tv.z;
                                acc.y += x2.y * tv.z;
                                acc.z += x2.z * tv.z;
                                acc.w += x2.w * tv.z;
                                acc2.x += x3.x * tv.w;
                                acc2.y += x3.y * tv.w;
                                acc2.z += x3.z * tv.w;
                                acc2.w += x3.w * tv.w;
                            }
                            acc.x += acc2.x;
                            acc.y += acc2.y;
                            acc.z += acc2.z;
                            acc.w += acc2.w;
                            if (part == 0) s1 = acc;
                            else s2 = acc;
                        }
                    }
                    // reduce-scatter over the 16 lanes: halve the eight sums at each
                    // exchange (row mirror, half-row mirror, then pairs), so that
                    // lanes 2k and 2k+1 end with sum 4 b3 + 2 b2 + b1 of the bits
                    // of k; the even lane writes it
                    const bool b3 = kq & 8, b2 = kq & 4, b1 = kq & 2;
                    const float v8[8] = {s1.x, s1.y, s1.z, s1.w, s2.x, s2.y, s2.z, s2.w};
                    float u4[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        u4[k] = (b3 ? v8[k + 4] : v8[k]) + dpp<kDppMirror16>(b3 ? v8[k] : v8[k + 4]);
                    float u2[2];
#pragma unroll
                    for (int k = 0; k < 2; ++k)
                        u2[k] = (b2 ? u4[k + 2] : u4[k]) + dpp<kDppMirror8>(b2 ? u4[k] : u4[k + 2]);
                    float z = (b1 ? u2[1] : u2[0]) + dpp<kDppXor2>(b1 ? u2[0] : u2[1]);
                    z += dpp<kDppXor1>(z);
                    if (!(kq & 1) && c1 <= c2) {
                        const int idx = (b3 ? 4 : 0) + (b2 ? 2 : 0) + (b1 ? 1 : 0);
                        const int j = 4 * (b3 ? c2 : c1) + (idx & 3);
                        if (j < m && (!b3 || c2 > c1)) vxn[j] = vx[j] + z;
                    }
                }
                __syncthreads();
                KAMX_MARK(3);
                // v~ - v~_f = D~ x_new (matrix-free, FP64): bodies gather here,
                // each block owner evaluates its own rows below
                delassus_gather_bal<NT>(L, nb, gnh, gorder, vp, vxn);
                KAMX_MARK(4);
                // steps 6-7 and the residuals of step 9 (block owners)
                float lrp = 0.f, lrd = 0.f, lrc = 0.f, lcc = 0.f;
                float yb[3], zb[3], xn[3], rr[3];
                // v~ - v~_f of row io in FP64: J_a M_a^-1 g_a on the even lane,
                // J_b M_b^-1 g_b on the odd lane, added by the pair sum
                {
                    double side = 0.0;
                    if (io < m) {
                        const int sb = hh == 0 ? L.ri(RIA, io) : L.ri(RIB, io);
                        if (sb >= 0) {
                            double wv[6];
                            body_minv64(L, sb, wv);
                            for (int c = 0; c < 6; ++c) side += (double)L.rf(RJ + 6 * hh + c, io) * wv[c];
                        }
                    }
                    side = lane_group_sum<2>(side);
                    if (hh == 0 && io < m) {
                        const double pr = (double)vp[io];
                        vdx[io] = (float)((side + (double)L.rf(RREG, io) * pr * (double)vxn[io]) * pr);
                    }
                }
                __syncthreads();
                if (owner_o) {
                    float zh[3], yh[3], ri[3], vv[3];
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        const float dx = vdx[io + e];
                        xn[e] = vxn[io + e];
                        zh[e] = vzh[io + e];
                        yh[e] = vyh[io + e];
                        rr[e] = e == 0 ? rho_o : vrho[io + e];
                        ri[e] = vrinv[io + e];
                        vv[e] = dx + vvt[io + e];
                    }
                    if (kind_o == kRowNormal) {
                        proj_cone(mu_o, xn[0] - zh[0] * ri[0], xn[1] - zh[1] * ri[1], xn[2] - zh[2] * ri[2], yb[0], yb[1],
                                  yb[2]);
                    } else if (kind_o == kRowLimit) {
                        yb[0] = fmaxf(xn[0] - zh[0] * ri[0], 0.f);
                    } else {
                        yb[0] = xn[0] - zh[0] * ri[0];
                    }
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        zb[e] = zh[e] - rr[e] * (xn[e] - yb[e]);
                        lrp = fmaxf(lrp, fabsf(xn[e] - yb[e]));
                        float dy = yb[e] - yh[e], dz = zb[e] - zh[e];
                        lcc += rr[e] * dy * dy + dz * dz * ri[e];
                    }
                    float g = kind_o == kRowNormal ? mu_o * hw_sqrt(vv[1] * vv[1] + vv[2] * vv[2]) : 0.f;
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        float d = vv[e] + (e == 0 ? g : 0.f) - zb[e];
                        lrd = fmaxf(lrd, fabsf(d));
                        if (d != d) lrd = d;
                    }
                    if (kind_o == kRowNormal) lrc = fabsf(yb[0] * (vv[0] + g) + yb[1] * vv[1] + yb[2] * vv[2]);
                    else if (kind_o == kRowLimit) lrc = fabsf(yb[0] * vv[0]);
                    if (lrp != lrp || lcc != lcc) lrp = NAN;
                }
                reduce4<NT>(lrp, lrd, lrc, lcc, L.red);
                rp = lrp;
                rd = lrd;
                rc = lrc;
                KAMX_MARK(5);
                // step 8: Nesterov with adaptive restart
                int restart = 0;
                float beta = 0.f;
                if (P.accel) {
                    restart = !(lcc < P.restart_factor * c_prev);
                    if (!restart) {
                        float a_next = 0.5f * (1.f + hw_sqrt(1.f + 4.f * a_k * a_k));
                        beta = (a_k - 1.f) * hw_rcp(a_next);
                        a_k = a_next;
                        c_prev = lcc;
                    } else {
                        a_k = 1.f;
                        c_prev = c_prev / P.restart_factor;
                    }
                }
                if (owner_o) {
                    float yn[3] = {0.f, 0.f, 0.f}, zn[3] = {0.f, 0.f, 0.f};
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        float yo = vyp[io + e], zo = vzp[io + e];
                        if (!P.accel) {
                            yn[e] = yb[e];
                            zn[e] = zb[e];
                        } else if (!restart) {
                            yn[e] = yb[e] + beta * (yb[e] - yo);
                            zn[e] = zb[e] + beta * (zb[e] - zo);
                        } else {
                            yn[e] = yo;
                            zn[e] = zo;
                        }
                        vyh[io + e] = yn[e];
                        vzh[io + e] = zn[e];
                        vx[io + e] = xn[e];
                        vyp[io + e] = yb[e];
                        vzp[io + e] = zb[e];
                    }
                    // the next right-hand side (as own_rhs) from the values in registers
                    s_own = kind_o == kRowNormal ? mu_o * hw_sqrt(zn[1] * zn[1] + zn[2] * zn[2]) : 0.f;
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        float rhs = -vvt[io + e] - (e == 0 ? s_own : 0.f) + eta * xn[e] + rr[e] * yn[e] + zn[e];
                        vrhs[io + e] = rhs - (vdx[io + e] + (eta + rr[e]) * xn[e]);
                    }
                }
                KAMX_MARK(6);
                // adaptive penalty (not in the paper: residual balancing) at the
                // checkpoints of a solve that does not exit here; rp and rd are
                // the same in every thread, so the branch is uniform
                int adapt_dir = 0;
                if (P.adapt_ratio > 0.f && n_uni > 0 && adapt_checkpoint(it, P.adapt_first) &&
                    !(P.fixed_iters <= 0 && rp < P.eps && rd < P.eps && rc < P.eps)) {
                    if (rd > P.adapt_ratio * rp) adapt_dir = 1;
                    else if (rp > P.adapt_ratio * rd) adapt_dir = 2;
                }
                if (tid == 0 && a.rlog && P.log_restarts && it <= P.max_iters)
                    a.rlog[(size_t)w * P.max_iters + (it - 1)] = (uint8_t)(restart | (adapt_dir << 1));
                if (!(isfinite(rp) && isfinite(rd) && isfinite(rc))) {
                    status = KAMX_WORLD_NONFINITE;
                    break;
                }
                if (P.fixed_iters <= 0 && rp < P.eps && rd < P.eps && rc < P.eps) {
                    converged = true;
                    break;
                }
                if (adapt_dir) {
                    adapt_pending = adapt_dir;
                    ++it;
                    break;
                }
            }
            if (!adapt_pending) break;
            {
                // the limit and contact rows' penalty changes by the factor;
                // D~ + diag(eta + rho) is rebuilt, refactored and inverted, and
                // the acceleration restarts at the current (y, z)
                const float f = adapt_pending == 1 ? 1.f / P.adapt_factor : P.adapt_factor;
                adapt_pending = 0;
                __syncthreads();
                for (int r = tid; r < m; r += NT)
                    if (L.ri(RKIND, r) != kRowBilateral) {
                        vrho[r] *= f;
                        vrinv[r] = 1.f / vrho[r];
                    }
                __syncthreads();
                reassemble<MC, NT>(L, A, m, nb, vp, vrho, eta);
                if (factor_invert_again<MC, NT>(L, A, m, s_int, a, w)) {
                    status = KAMX_WORLD_FACTOR_FAIL;
                    break;
                }
                rho_o = io < m ? vrho[io] : 1.f;
                a_k = 1.f;
                c_prev = INFINITY;
                if (owner_o) {
                    _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk_o) {
                        vyh[io + e] = vyp[io + e];
                        vzh[io + e] = vzp[io + e];
                    }
                }
                __syncthreads();
                own_rhs();
            }
        }
#undef KAMX_MARK
#ifndef KAMX_FACTOR_TIMING
        if (timing)
            for (int k = 0; k < 6; ++k) a.phase_clk[16 * w + 8 + k] = sub[k];
#endif
        if (it > N) it = N;
        if (P.fixed_iters <= 0 && !converged && status == 0) status = KAMX_WORLD_MAXITER;
        __syncthreads();
        // natural-map residual of the NCP at the returned y (Eq. 3)
        delassus_apply<NT>(L, m, nb, vp, vyp, vaux);
        float lncp = 0.f;
        if (owner) {
            float v[3], o[3], y[3], nm[3];
            _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk) {
                v[e] = vaux[i + e] + vvt[i + e];
                y[e] = vyp[i + e];
            }
            float g = kind_i == kRowNormal ? mu_i * sqrtf(v[1] * v[1] + v[2] * v[2]) : 0.f;
            _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk) nm[e] = y[e] - (v[e] + (e == 0 ? g : 0.f));
            if (kind_i == kRowNormal) proj_cone(mu_i, nm[0], nm[1], nm[2], o[0], o[1], o[2]);
            else if (kind_i == kRowLimit) o[0] = fmaxf(nm[0], 0.f);
            else o[0] = nm[0];
            _Pragma("unroll") for (int e = 0; e < 3; ++e) if (e < blk) lncp = fmaxf(lncp, fabsf(y[e] - o[e]));
        }
        float l1 = 0.f, l2 = 0.f, l3 = 0.f;
        reduce4<NT>(lncp, l1, l2, l3, L.red);
        rncp = lncp;
    }
    __syncthreads();

    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 6] = wall_clock64();
    // ---- outputs: lambda = P y (Alg. 1 step 11), stats, caches
    if (i < W.row_cap) {
        float lam = 0.f;
        if (i < m) lam = vp[i] * vyp[i];
        a.lambda[W.row_base + i] = lam;
        if (i < m) vaux[i] = lam;
        if (a.iterate_out) {
            // the returned iterate in preconditioned units and the scales
            const bool act = i < m;
            *reinterpret_cast<float4 *>(a.iterate_out + 4 * ((long)W.row_base + i)) =
                make_float4(act ? vx[i] : 0.f, act ? vyp[i] : 0.f, act ? vzp[i] : 0.f, act ? vp[i] : 0.f);
        }
    }
    if (tid == 0) {
        a.iters[w] = it;
        a.status[w] = status;
        if (a.iter_log && k < a.iter_log_rows) {
            a.iter_log[(long)k * a.n_worlds + w] = it;
            if (a.row_log) a.row_log[(long)k * a.n_worlds + w] = m;
            if (a.status_log) a.status_log[(long)k * a.n_worlds + w] = status;
        }
        a.rows[w] = m;
        a.resid[4 * w + 0] = rp;
        a.resid[4 * w + 1] = rd;
        a.resid[4 * w + 2] = rc;
        a.resid[4 * w + 3] = rncp;
        a.ncontacts_out[w] = nc;
    }
    for (int c = tid; c < nc; c += NT) {
        kamx_contact ct;
        ct.body_a = cint[CA * kMaxContacts + c] + W.b0;
        int lb = cint[CB * kMaxContacts + c];
        ct.body_b = lb >= 0 ? lb + W.b0 : -1;
        for (int k = 0; k < 3; ++k) {
            ct.point[k] = L.cf(CP + k, c);
            ct.normal[k] = L.cf(CN + k, c);
        }
        ct.gap = L.cf(CGAP, c);
        ct.mu = L.cf(CMU, c);
        ct.key = cint[CKEY * kMaxContacts + c];
        a.contacts_out[w * kMaxContacts + c] = ct;
        a.keys[w * kMaxContacts + c] = ct.key;
    }
    __syncthreads();

    // ---- u+ = u_f + M^-1 J^T lambda (FP64 accumulation over the incident
    //      rows: light links carry large, nearly cancelling impulses), then
    //      poses by the exponential map
    for (int b = tid; b < nb; b += NT) {
        double imp[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = L.inc_off[b]; k < L.inc_off[b + 1]; ++k) {
            int e = L.inc_list[k];
            int r = e >> 1, side = e & 1;
            double lam = (double)vp[r] * (double)vyp[r];
            if (factor_fail) lam = 0.0;
            for (int c = 0; c < 6; ++c) imp[c] += (double)L.rf(RJ + 6 * side + c, r) * lam;
        }
        double R[9], t[3], sv[3];
        for (int c = 0; c < 9; ++c) R[c] = L.bf(BR + c, b);
        mtv3(R, imp + 3, t);
        for (int c = 0; c < 3; ++c) t[c] *= (double)L.bf(BII + c, b);
        mv3(R, t, sv);
        double im = L.bf(BIM, b);
        float un[6];
        for (int c = 0; c < 3; ++c) {
            un[c] = (float)((double)L.bf(BUF + c, b) + imp[c] * im);
            un[3 + c] = (float)((double)L.bf(BUF + 3 + c, b) + sv[c]);
        }
        int gb = W.b0 + b;
        for (int k = 0; k < 6; ++k) a.u[6 * gb + k] = un[k];
        // poses over the rest of the step from the rows' configuration: dt
        // (Euler) or dt / 2 from the half-step poses (Moreau-Jean)
        double q[7], ud[6], qn[7];
        for (int k = 0; k < 7; ++k) q[k] = L.qd[k * kMaxBodies + b];
        for (int k = 0; k < 6; ++k) ud[k] = un[k];
        advance_pose(q, ud, (P.integrator == KAMX_MOREAU_JEAN ? 0.5 : 1.0) * (double)P.dt, qn);
        for (int k = 0; k < 7; ++k) a.q[7 * gb + k] = (float)qn[k];
    }
    __syncthreads();
    if (a.phase_clk && tid == 0) a.phase_clk[16 * w + 7] = wall_clock64();
}

// A launch advances every world of the bucket by a.nsteps steps, the
// workgroup keeping its world for all of them: worlds are independent, so a
// slow solve delays only its own world and the hardware's dispatch balances
// whole chains of steps rather than single steps.
// At most 256 VGPRs (two waves per SIMD): the per-step function needs 248,
// and a workgroup smaller than 512 threads then leaves room on its compute
// unit for another world's workgroup.
template <int MC, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void step_kernel(StepArgs a) {
    __shared__ int s_int[8];
    // the arguments in LDS: the per-step function takes them by reference,
    // which would otherwise copy them to every lane's private stack
    __shared__ StepArgs sa;
    if (threadIdx.x == 0) sa = a;
    __syncthreads();
#pragma clang loop unroll(disable)
    for (int k = 0; k < sa.nsteps; ++k) {
        step_world<MC, NT>(sa, k, s_int);
        __syncthreads();
    }
}

// Impulses of the last step in slot layout (joint, limit and drive rows, then three
// slots per contact key; slots of absent contacts are zero), one thread per
// world and slot.
__global__ void impulse_slots_kernel(const WorldInfo *worlds, int n_worlds, int n_contact_slots, const float *lambda,
                                     const int32_t *keys, const int32_t *ncontacts, float *out) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const WorldInfo W0 = worlds[0];
    const int S = 5 * W0.nj + W0.nlim + W0.ndrv + 3 * n_contact_slots;
    if (idx >= (long)n_worlds * S) return;
    const int w = (int)(idx / S), t = (int)(idx - (long)w * S);
    const WorldInfo W = worlds[w];
    const int rc0 = 5 * W.nj + W.nlim + W.ndrv;
    float v = 0.f;
    if (t < rc0) {
        v = lambda[W.row_base + t];
    } else {
        const int slot = (t - rc0) / 3, e = (t - rc0) % 3;
        const int n = ncontacts[w];
        for (int k = 0; k < n && k < kMaxContacts; ++k)
            if (keys[w * kMaxContacts + k] >= 0 && contact_slot(keys[w * kMaxContacts + k]) == slot) {
                v = lambda[W.row_base + rc0 + 3 * k + e];
                break;
            }
    }
    out[idx] = v;
}

hipError_t launch_impulse_slots(const WorldInfo *worlds, int n_worlds, int n_contact_slots, int n_slots,
                                const float *lambda, const int32_t *keys, const int32_t *ncontacts, float *out,
                                hipStream_t stream) {
    const long total = (long)n_worlds * n_slots;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(impulse_slots_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, worlds,
                       n_worlds, n_contact_slots, lambda, keys, ncontacts, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launch table
// ---------------------------------------------------------------------------

template <int MC, int NT>
static hipError_t launch_mc(const StepArgs &args, int n, hipStream_t stream) {
    static_assert(NT % 64 == 0 && NT >= 64 && NT >= 2 * MC && NT <= 512, "unsupported workgroup size");
    size_t bytes = sizeof(float) * (size_t)smem_floats(MC);
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)step_kernel<MC, NT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
        configured = true;
    }
    hipLaunchKernelGGL((step_kernel<MC, NT>), dim3(n), dim3(NT), bytes, stream, args);
    return hipGetLastError();
}

int bucket_capacity(int rows) {
    static const int caps[] = {32, 64, 96, 128, 160, 192, 224};
    for (int c : caps)
        if (rows <= c) return c;
    return -1;
}

// Workgroup sizes each row bucket is built for.  Every iteration pass gives
// each pair of rows (and each pair of column quads) its own threads, so a
// workgroup has at least two threads per row; the larger size runs the
// passes with more threads, the smaller one lets more worlds share a compute
// unit where LDS allows.  The 32-row bucket also runs one wavefront per
// world (its 16x16 tile factorization needs no second wave: the trailing
// update of two tiles is the next diagonal tile, which wave 0 takes).  The first entry is the
// default.  Results do not depend on the choice: every row, tile and
// reduction is evaluated in the same order at every size.
int step_threads_variants(int mc, int out[4]) {
    if (mc == 256 || mc == 512 || mc == 1024) {  // matrix-free: one thread per row
        out[0] = mc;
        return 1;
    }
    for (const BucketSizes &v : kBucketSizes)  // 32 rows: 64 is one wavefront per world
        if (v.mc == mc) {
            for (int k = 0; k < v.n; ++k) out[k] = v.nt[k];
            return v.n;
        }
    return 0;
}

hipError_t launch_sparse_step(const StepArgs &args, int nt, int n, hipStream_t stream);
size_t sparse_smem_bytes(int nt);

hipError_t launch_step(const StepArgs &args, int mc, int nt, int n, hipStream_t stream) {
    if (mc > kMaxRows) return launch_sparse_step(args, nt, n, stream);  // matrix-free row classes
    switch (mc * 1024 + nt) {
    case 32 * 1024 + 64: return launch_mc<32, 64>(args, n, stream);
    case 32 * 1024 + 128: return launch_mc<32, 128>(args, n, stream);
    case 32 * 1024 + 256: return launch_mc<32, 256>(args, n, stream);
    case 64 * 1024 + 128: return launch_mc<64, 128>(args, n, stream);
    case 64 * 1024 + 256: return launch_mc<64, 256>(args, n, stream);
    case 96 * 1024 + 256: return launch_mc<96, 256>(args, n, stream);
    case 96 * 1024 + 512: return launch_mc<96, 512>(args, n, stream);
    case 128 * 1024 + 256: return launch_mc<128, 256>(args, n, stream);
    case 128 * 1024 + 512: return launch_mc<128, 512>(args, n, stream);
    case 160 * 1024 + 384: return launch_mc<160, 384>(args, n, stream);
    case 160 * 1024 + 512: return launch_mc<160, 512>(args, n, stream);
    case 192 * 1024 + 384: return launch_mc<192, 384>(args, n, stream);
    case 192 * 1024 + 512: return launch_mc<192, 512>(args, n, stream);
    case 224 * 1024 + 512: return launch_mc<224, 512>(args, n, stream);
    default: return hipErrorInvalidValue;
    }
}

size_t step_smem_bytes(int mc) { return mc > kMaxRows ? sparse_smem_bytes(mc) : sizeof(float) * (size_t)smem_floats(mc); }

// whether the step kernel of a row bucket can generate box-bin contacts
// itself (the candidates must fit in the LDS of its Delassus triangle)
bool step_generates_box_contacts(int mc) {
    return mc <= kMaxRows && sizeof(float) * (size_t)tri_row_offset(mc) >= sizeof(BoxLds);
}

}  // namespace kamx
