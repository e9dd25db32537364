// Matrix-free per-world time step for large worlds (Sec. 5.1, the sparse
// formulation): the Delassus operator is never formed.  Its product with a
// vector is evaluated through the constraint Jacobian with the mass matrix
// and the preconditioner folded in once per step ("pre-baked"):
//
//   J~_r,b = p_r J_r,b M_b^-1/2     (a 6-vector per row and side)
//   D~ v   = J~ (J~^T v) + P R P v  (R: drive-row regularisation, Eq. 4)
//
// and the x-update of Alg. 1 step 5 is a Conjugate Residual solve with a
// fixed budget, warm-started at the previous iterate (Sec. 4.1, Sec. 5.1).
//
// One workgroup per world, one constraint row per thread.  A row's data
// (its J~ 6-blocks, scale, penalty, kind and every ADMM and CR vector entry)
// stays in the registers of its thread for the whole step; only what other
// threads read goes through LDS: J~ and the vector being multiplied (read by
// the body gather), the per-body gather sums (read by the rows) and the
// per-wave partial sums of the reductions.  A product D~ v costs one body
// gather (one thread per body and component, FP64 accumulation over the
// body's incident rows in increasing row order) and one row evaluation (FP64
// over the row's two 6-blocks), with a workgroup barrier after each.
//
// Rows: joint rows (5 per joint), limit rows, drive rows, then contacts.  A
// contact's rows (n, t1, t2) occupy the first three lanes of an aligned
// group of four lanes (the fourth idles), so the cone projection, the De
// Saxce term and the complementarity product exchange a contact's entries
// by DPP quad permutations, with no LDS traffic and no owner thread.
#include <math.h>

#include "kamx_device.h"
#include "kamx_geom.h"
#include "kamx_internal.h"

namespace kamx {

constexpr int kSpBodies = KAMX_MAX_BODIES_SPARSE;
constexpr int kSpJoints = KAMX_MAX_JOINTS_SPARSE;

// body fields [field][kSpBodies] (the dense kernel's order)
enum { SBQ = 0, SBU = 7, SBUF = 13, SBR = 19, SBII = 28, SBIM = 31 };
// joint fields [field][kSpJoints]
enum { SJTAU = 0, SJC = 1, SJA = 13, SJB = 14, SJTF = 15 };
// contact fields [field][kMaxContacts]
enum { SCP = 0, SCN = 3, SCGAP = 6, SCMU = 7, SCA = 8, SCB = 9, SCKEY = 10 };
// row scratch fields [field][NT] (filled by the joint and contact threads,
// read once by the row threads)
enum { SRBIAS = 0, SRMU = 1, SRREG = 2, SRKIND = 3 };

constexpr int kRowPad = -1;  // an inactive row (alignment padding, or past the world's rows)

// LDS footprint in floats for a workgroup of NT threads (doubles first)
__host__ __device__ constexpr int sp_smem_floats(int nt) {
    return 2 * 7 * kSpBodies + 2 * 6 * kSpBodies        // FP64 poses, FP64 gather sums
           + 32 * kSpBodies + 16 * kSpJoints + 12 * kMaxContacts
           + 12 * nt + 4 * nt + nt + nt                // J~, row scratch, row bodies, vector
           + (((kSpBodies + 1 + 2 * nt) + 3) & ~3)    // incidence lists
           + 128;                                      // reduction partials (two buffers)
}

struct SpLds {
    double *qd;   // [7][kSpBodies] poses the rows are built at (FP64)
    double *g;    // [6][kSpBodies] body gather sums of the last product (FP64)
    float *b;     // [32][kSpBodies]
    float *j;     // [16][kSpJoints]
    float *c;     // [12][kMaxContacts]
    float *J;     // [12][nt] raw rows, then J~
    float *rs;    // [4][nt] row scratch
    int *rab;     // [nt] (a + 1) | (b + 1) << 16, 0: none
    float *v;     // [nt] the vector of the current product
    int *inc_off;   // [kSpBodies + 1]
    int *inc_list;  // [2 nt] (row << 1) | side
    float *red;   // [2][16 waves][4]
    int nt;
    __device__ float &bf(int f, int i) const { return b[f * kSpBodies + i]; }
    __device__ float &jfld(int f, int i) const { return j[f * kSpJoints + i]; }
    __device__ int &ji(int f, int i) const { return reinterpret_cast<int *>(j)[f * kSpJoints + i]; }
    __device__ float &cf(int f, int i) const { return c[f * kMaxContacts + i]; }
    __device__ int &ci(int f, int i) const { return reinterpret_cast<int *>(c)[f * kMaxContacts + i]; }
    __device__ float &rf(int f, int r) const { return rs[f * nt + r]; }
    __device__ int &ri(int f, int r) const { return reinterpret_cast<int *>(rs)[f * nt + r]; }
};

// Broadcast of quad lane K to the four lanes of its aligned quad (DPP quad
// permutation); every lane of the wave must be active.
template <int K>
__device__ inline float quad_bc(float v) {
    return dpp<K * 0x55>(v);
}

// Sums over the workgroup of up to four per-thread values (fixed order: DPP
// rows of 16, readlane across the wave, waves in index order through LDS;
// every thread ends with the same bits).  buf alternates between two
// halves of red, so consecutive reductions need one barrier each.
template <int NT, int NV>
__device__ inline void sp_sum(float (&s)[4], float *red, int &buf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *rb = red + 64 * buf;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        float v = lane_group_sum<16>(s[k]);
        v = (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
        if (lane == 0) rb[4 * wave + k] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        float acc = rb[k];
        for (int q = 1; q < NT / 64; ++q) acc += rb[4 * q + k];
        s[k] = acc;
    }
    buf ^= 1;
}

// Maxima (m0..m2, values >= +0 or NaN) and one sum (s3) over the workgroup.
template <int NT>
__device__ inline void sp_max3_sum(float &m0, float &m1, float &m2, float &s3, float *red, int &buf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *rb = red + 64 * buf;
    m0 = lane_group_max<16>(m0);
    m1 = lane_group_max<16>(m1);
    m2 = lane_group_max<16>(m2);
    s3 = lane_group_sum<16>(s3);
    m0 = max_nonneg(max_nonneg(rdlane(m0, 0), rdlane(m0, 16)), max_nonneg(rdlane(m0, 32), rdlane(m0, 48)));
    m1 = max_nonneg(max_nonneg(rdlane(m1, 0), rdlane(m1, 16)), max_nonneg(rdlane(m1, 32), rdlane(m1, 48)));
    m2 = max_nonneg(max_nonneg(rdlane(m2, 0), rdlane(m2, 16)), max_nonneg(rdlane(m2, 32), rdlane(m2, 48)));
    s3 = (rdlane(s3, 0) + rdlane(s3, 16)) + (rdlane(s3, 32) + rdlane(s3, 48));
    if (lane == 0) {
        rb[4 * wave + 0] = m0;
        rb[4 * wave + 1] = m1;
        rb[4 * wave + 2] = m2;
        rb[4 * wave + 3] = s3;
    }
    __syncthreads();
    m0 = rb[0];
    m1 = rb[1];
    m2 = rb[2];
    s3 = rb[3];
    for (int q = 1; q < NT / 64; ++q) {
        m0 = max_nonneg(m0, rb[4 * q]);
        m1 = max_nonneg(m1, rb[4 * q + 1]);
        m2 = max_nonneg(m2, rb[4 * q + 2]);
        s3 = s3 + rb[4 * q + 3];
    }
    buf ^= 1;
}

// The register-resident part of a row.
struct SpRow {
    int kind;      // kRowBilateral, kRowLimit, kRowNormal, kRowTangent, or kRowPad
    int a, b;      // world-local bodies (b = -1: the world)
    float jt[12];  // J~ (both sides)
    float preg;    // p^2 R (drive rows), else 0
};

// M_b^-1/2 applied to a 6-vector in the body frame: lin / sqrt(m),
// R diag(I^-1/2) R^T ang
__device__ inline void half_inv_mass(const SpLds &L, int b, const float in[6], float out[6]) {
    const float sm = sqrtf(L.bf(SBIM, b));
    for (int k = 0; k < 3; ++k) out[k] = in[k] * sm;
    float R[9], t[3], s[3];
    for (int k = 0; k < 9; ++k) R[k] = L.bf(SBR + k, b);
    mtv3(R, in + 3, t);
    for (int k = 0; k < 3; ++k) t[k] *= sqrtf(L.bf(SBII + k, b));
    mv3(R, t, s);
    for (int k = 0; k < 3; ++k) out[3 + k] = s[k];
}

// One product D~ v: thread t contributes v_t (0 on inactive rows and
// threads); returns (D~ v)_t.  The body gather sums J~_b^T v (FP64) stay in
// L.g until the next product.  Two barriers.
template <int NT>
__device__ inline float sp_apply(const SpLds &L, const SpRow &R, int nb, float vt) {
    const int tid = threadIdx.x;
    L.v[tid] = vt;
    __syncthreads();
    for (int task = tid; task < 6 * nb; task += NT) {
        const int bb = task / 6, c = task - 6 * (task / 6);
        double acc = 0.0;
        const int k1 = L.inc_off[bb + 1];
        for (int k = L.inc_off[bb]; k < k1; ++k) {
            const int e = L.inc_list[k];
            const int r = e >> 1;
            acc += (double)L.J[(6 * (e & 1) + c) * NT + r] * (double)L.v[r];
        }
        L.g[c * kSpBodies + bb] = acc;
    }
    __syncthreads();
    double out = 0.0;
    if (R.kind != kRowPad) {
        for (int c = 0; c < 6; ++c) out += (double)R.jt[c] * L.g[c * kSpBodies + R.a];
        if (R.b >= 0)
            for (int c = 0; c < 6; ++c) out += (double)R.jt[6 + c] * L.g[c * kSpBodies + R.b];
        out += (double)R.preg * (double)vt;
    }
    return (float)out;
}

// Pi_K of a row's entry of w (Alg. 1 step 6): identity on bilateral rows,
// max(0, .) on limit rows, the Coulomb cone on a contact's quad.  Every
// lane of the wave must call it (quad permutations).
__device__ inline float sp_project(const SpRow &R, float mu, int e, float w) {
    const float w0 = quad_bc<0>(w), w1 = quad_bc<1>(w), w2 = quad_bc<2>(w);
    if (R.kind == kRowNormal || R.kind == kRowTangent) {
        float o0, o1, o2;
        proj_cone(mu, w0, w1, w2, o0, o1, o2);
        return e == 0 ? o0 : (e == 1 ? o1 : o2);
    }
    if (R.kind == kRowLimit) return fmaxf(w, 0.f);
    if (R.kind == kRowPad) return 0.f;
    return w;
}

// The De Saxce term Gamma(w) of a row (mu ||w_t|| on a contact's normal
// row, 0 elsewhere); every lane must call it.
__device__ inline float sp_gamma(const SpRow &R, float mu, float w) {
    const float w1 = quad_bc<1>(w), w2 = quad_bc<2>(w);
    return R.kind == kRowNormal ? mu * sqrtf(w1 * w1 + w2 * w2) : 0.f;
}

template <int NT>
__device__ __attribute__((noinline)) void sparse_step_world(const StepArgs &a, int k, int *s_int) {
    extern __shared__ float4 smem4[];
    float *sm = reinterpret_cast<float *>(smem4);
    const int tid = threadIdx.x;
    const int w = a.bucket_worlds[blockIdx.x];
    const uint32_t step = *a.step_ctr + (uint32_t)k;
    const WorldInfo W = a.worlds[w];
    const SolverParams &P = a.p;

    SpLds L;
    L.nt = NT;
    L.qd = reinterpret_cast<double *>(sm);
    L.g = L.qd + 7 * kSpBodies;
    L.b = reinterpret_cast<float *>(L.g + 6 * kSpBodies);
    L.j = L.b + 32 * kSpBodies;
    L.c = L.j + 16 * kSpJoints;
    L.J = L.c + 12 * kMaxContacts;
    L.rs = L.J + 12 * NT;
    L.rab = reinterpret_cast<int *>(L.rs + 4 * NT);
    L.v = reinterpret_cast<float *>(L.rab + NT);
    L.inc_off = reinterpret_cast<int *>(L.v + NT);
    L.inc_list = L.inc_off + kSpBodies + 1;
    L.red = reinterpret_cast<float *>(L.inc_off + (((kSpBodies + 1 + 2 * NT) + 3) & ~3));
    int rbuf = 0;

    const int nb = W.nb, nj = W.nj;

    // ---- reset: a world whose reset body fell below the threshold restarts
    if (tid == 0) {
        int rs = 0;
        if (W.reset_body >= 0) rs = a.q[7 * (W.b0 + W.reset_body) + 2] < P.reset_height;
        s_int[0] = rs;
        if (rs && a.stage == 0) a.reset_count[w] += 1;
    }
    __syncthreads();
    const int reset = s_int[0];
    if (a.stage == 1) return;  // no feature vector for matrix-free worlds

    // ---- bodies (Sec. 3, Eq. 1): state, rotation, inverse mass properties;
    //      the configuration the rows are built at in FP64 (the pre-step
    //      pose, or the Moreau-Jean half step)
    for (int bb = tid; bb < nb; bb += NT) {
        const int gb = W.b0 + bb;
        const float *qs = reset ? a.q0 : a.q;
        const float *us = reset ? a.u0 : a.u;
        float q[7], u6[6];
        for (int e = 0; e < 7; ++e) q[e] = qs[7 * gb + e];
        for (int e = 0; e < 6; ++e) u6[e] = us[6 * gb + e];
        double qd[7];
        for (int e = 0; e < 7; ++e) qd[e] = q[e];
        if (P.integrator == KAMX_MOREAU_JEAN) {
            double u6d[6], qm[7];
            for (int e = 0; e < 6; ++e) u6d[e] = u6[e];
            advance_pose(qd, u6d, 0.5 * (double)P.dt, qm);
            for (int e = 0; e < 7; ++e) {
                qd[e] = qm[e];
                q[e] = (float)qm[e];
            }
        }
        for (int e = 0; e < 7; ++e) L.qd[e * kSpBodies + bb] = qd[e];
        for (int e = 0; e < 7; ++e) L.bf(SBQ + e, bb) = q[e];
        for (int e = 0; e < 6; ++e) L.bf(SBU + e, bb) = u6[e];
        float Rm[9];
        rot_of_quat(q + 3, Rm);
        for (int e = 0; e < 9; ++e) L.bf(SBR + e, bb) = Rm[e];
        for (int e = 0; e < 3; ++e) L.bf(SBII + e, bb) = 1.f / a.inertia[3 * gb + e];
        L.bf(SBIM, bb) = 1.f / a.mass[gb];
    }
    __syncthreads();

    // ---- joints: coordinate, rate and actuation along the coordinate
    //      (external + explicit PD + noise)
    for (int j = tid; j < nj; j += NT) {
        const int gj = W.j0 + j;
        const int type = a.jint[4 * gj], la = a.jint[4 * gj + 1], lb = a.jint[4 * gj + 2], fl = a.jint[4 * gj + 3];
        const float *jf = a.jf + kJointFloats * gj;
        double qa[7], qb[7];
        for (int e = 0; e < 7; ++e) qa[e] = L.qd[e * kSpBodies + la];
        for (int e = 0; e < 7; ++e) qb[e] = lb >= 0 ? L.qd[e * kSpBodies + lb] : 0.0;
        JointGeo g;
        joint_geo_q(qa, qb, lb >= 0, jf, g);
        float Ja[6], Jb[6];
        const float c = (float)joint_coord(type, g, Ja, Jb);
        float rate = 0.f;
        for (int e = 0; e < 6; ++e) rate += Ja[e] * L.bf(SBU + e, la);
        if (lb >= 0)
            for (int e = 0; e < 6; ++e) rate += Jb[e] * L.bf(SBU + e, lb);
        float tau = a.ext_tau ? a.ext_tau[gj] : 0.f;
        const float kp = jf[16], kd = jf[17], ref = jf[18];
        if (!(fl & kJointDriven) && (kp != 0.f || kd != 0.f)) tau += kp * (ref - c) - kd * rate;
        if ((fl & kJointActuated) && P.torque_sigma != 0.f)
            tau += P.torque_sigma * noise_normal(P.seed_lo, P.seed_hi, (uint32_t)w, step, (uint32_t)j);
        L.jfld(SJTAU, j) = tau;
        for (int e = 0; e < 6; ++e) {
            L.jfld(SJC + e, j) = Ja[e];
            L.jfld(SJC + 6 + e, j) = Jb[e];
        }
        L.ji(SJA, j) = la;
        L.ji(SJB, j) = lb;
        L.ji(SJTF, j) = type | (fl << 4);
        a.tau_out[gj] = tau;
    }
    __syncthreads();

    // ---- free velocity u_f = u + dt M^-1 h (gravity, gyroscopic term, joint
    //      actuation)
    for (int bb = tid; bb < nb; bb += NT) {
        const float m = 1.f / L.bf(SBIM, bb);
        float h[6];
        h[0] = m * P.gx;
        h[1] = m * P.gy;
        h[2] = m * P.gz;
        float Rm[9], w3[3], t[3], Iw[3], gyro[3];
        for (int e = 0; e < 9; ++e) Rm[e] = L.bf(SBR + e, bb);
        for (int e = 0; e < 3; ++e) w3[e] = L.bf(SBU + 3 + e, bb);
        mtv3(Rm, w3, t);
        for (int e = 0; e < 3; ++e) t[e] /= L.bf(SBII + e, bb);
        mv3(Rm, t, Iw);
        cross(w3, Iw, gyro);
        h[3] = -gyro[0];
        h[4] = -gyro[1];
        h[5] = -gyro[2];
        for (int j = 0; j < nj; ++j) {
            const float tau = L.jfld(SJTAU, j);
            if (tau == 0.f) continue;
            if (L.ji(SJA, j) == bb)
                for (int e = 0; e < 6; ++e) h[e] += tau * L.jfld(SJC + e, j);
            if (L.ji(SJB, j) == bb)
                for (int e = 0; e < 6; ++e) h[e] += tau * L.jfld(SJC + 6 + e, j);
        }
        // M^-1 h in the body frame
        const float im = L.bf(SBIM, bb);
        float s[3];
        mtv3(Rm, h + 3, t);
        for (int e = 0; e < 3; ++e) t[e] *= L.bf(SBII + e, bb);
        mv3(Rm, t, s);
        for (int e = 0; e < 3; ++e) {
            L.bf(SBUF + e, bb) = L.bf(SBU + e, bb) + P.dt * (h[e] * im);
            L.bf(SBUF + 3 + e, bb) = L.bf(SBU + 3 + e, bb) + P.dt * s[e];
        }
    }

    // ---- contacts: explicit list (uploaded or generated before the step),
    //      or probes below the margin compacted in probe order
    if (a.contacts) {
        const int c0 = a.ccount ? w * kMaxContacts : a.coff[w];
        int n = a.ccount ? a.ccount[w] : a.coff[w + 1] - c0;
        if (n > W.contact_cap) n = W.contact_cap;
        if (n < 0) n = 0;
        if (tid == 0) s_int[1] = n;
        for (int c = tid; c < n; c += NT) {
            const kamx_contact ct = a.contacts[c0 + c];
            const int la = ct.body_a - W.b0;
            const int lb = ct.body_b < 0 ? -1 : ct.body_b - W.b0;
            const bool ok = la >= 0 && la < nb && lb < nb;
            for (int e = 0; e < 3; ++e) {
                L.cf(SCP + e, c) = ct.point[e];
                L.cf(SCN + e, c) = ct.normal[e];
            }
            L.cf(SCGAP, c) = ok ? ct.gap : 1e30f;  // an invalid contact becomes inert
            L.cf(SCMU, c) = ct.mu;
            L.ci(SCA, c) = ok ? la : 0;
            L.ci(SCB, c) = ok ? lb : -1;
            L.ci(SCKEY, c) = ct.key;
        }
    } else if (tid < 64) {
        const int kp = tid;
        bool act = false;
        float pw[3] = {0.f, 0.f, 0.f};
        int lbod = 0;
        float mu = 0.f;
        if (kp < W.np) {
            const int gp = W.p0 + kp;
            lbod = a.pbody[gp];
            mu = a.pf[4 * gp + 3];
            double qq[4], Rd[9], pld[3] = {a.pf[4 * gp], a.pf[4 * gp + 1], a.pf[4 * gp + 2]}, td[3];
            for (int e = 0; e < 4; ++e) qq[e] = L.qd[(3 + e) * kSpBodies + lbod];
            rot_of_quat(qq, Rd);
            mv3(Rd, pld, td);
            for (int e = 0; e < 3; ++e) pw[e] = (float)(L.qd[e * kSpBodies + lbod] + td[e]);
            act = pw[2] < P.contact_margin;
        }
        const unsigned long long mask = __ballot(act);
        const int slot = __popcll(mask & ((1ull << kp) - 1ull));
        if (act && slot < W.contact_cap) {
            for (int e = 0; e < 3; ++e) L.cf(SCP + e, slot) = pw[e];
            L.cf(SCN + 0, slot) = 0.f;
            L.cf(SCN + 1, slot) = 0.f;
            L.cf(SCN + 2, slot) = 1.f;
            L.cf(SCGAP, slot) = pw[2];
            L.cf(SCMU, slot) = mu;
            L.ci(SCA, slot) = lbod;
            L.ci(SCB, slot) = -1;
            L.ci(SCKEY, slot) = kp;
        }
        if (kp == 0) {
            const int n = __popcll(mask);
            s_int[1] = n < W.contact_cap ? n : W.contact_cap;
        }
    }
    __syncthreads();
    const int nc = s_int[1];
    const int row_lim0 = 5 * nj;
    const int row_drv0 = row_lim0 + W.nlim;
    const int row_c0 = row_drv0 + W.ndrv;   // first contact row (compact order)
    const int rc0p = (row_c0 + 3) & ~3;     // first contact quad (thread order)
    const int m_int = rc0p + 4 * nc;        // threads with a row or a pad
    const int m = row_c0 + 3 * nc;          // active rows

    // ---- constraint rows (Sec. 3): raw J in L.J, bias / mu / R / kind in
    //      the row scratch, bodies in L.rab
    auto put_row = [&](int r, const float Ja[6], int la, const float Jb[6], int lb, float f, int kind, float mu) {
        for (int e = 0; e < 6; ++e) {
            L.J[e * NT + r] = Ja[e];
            L.J[(6 + e) * NT + r] = lb >= 0 ? Jb[e] : 0.f;
        }
        L.rab[r] = (la + 1) | ((lb + 1) << 16);
        L.ri(SRKIND, r) = kind;
        L.rf(SRMU, r) = mu;
        L.rf(SRREG, r) = 0.f;
        const float inv_h = (P.integrator == KAMX_MOREAU_JEAN ? 2.f : 1.f) / P.dt;
        float bias = 0.f;
        if (kind == kRowBilateral) bias = P.baumgarte * f * inv_h;
        else if (kind == kRowLimit || kind == kRowNormal) bias = (f >= 0.f ? f : P.baumgarte * f) * inv_h;
        L.rf(SRBIAS, r) = bias;
    };
    for (int r = row_c0 + tid; r < NT; r += NT) {
        // padding rows between the compact rows and the contact quads, and
        // past the last quad
        const bool quad_lane = r >= rc0p && r < m_int && ((r - rc0p) & 3) != 3;
        if (!quad_lane) {
            L.ri(SRKIND, r) = kRowPad;
            L.rab[r] = 0;
            for (int e = 0; e < 12; ++e) L.J[e * NT + r] = 0.f;
            L.rf(SRBIAS, r) = 0.f;
            L.rf(SRMU, r) = 0.f;
            L.rf(SRREG, r) = 0.f;
        }
    }
    for (int j = tid; j < nj; j += NT) {
        const int gj = W.j0 + j;
        const int type = a.jint[4 * gj], la = a.jint[4 * gj + 1], lb = a.jint[4 * gj + 2], fl = a.jint[4 * gj + 3];
        const float *jf = a.jf + kJointFloats * gj;
        double qa[7], qb[7];
        for (int e = 0; e < 7; ++e) qa[e] = L.qd[e * kSpBodies + la];
        for (int e = 0; e < 7; ++e) qb[e] = lb >= 0 ? L.qd[e * kSpBodies + lb] : 0.0;
        JointGeo g;
        joint_geo_q(qa, qb, lb >= 0, jf, g);
        joint_constraints(type, g, [&](int e, const double Jad[6], const double Jbd[6], double f) {
            float fa[6], fb[6];
            for (int q = 0; q < 6; ++q) {
                fa[q] = (float)Jad[q];
                fb[q] = (float)Jbd[q];
            }
            put_row(5 * j + e, fa, la, fb, lb, (float)f, kRowBilateral, 0.f);
        });
        if (fl & kJointLimited) {
            int rank = 0;
            for (int q = 0; q < j; ++q) rank += (L.ji(SJTF, q) >> 4) & kJointLimited ? 1 : 0;
            float Ja[6], Jb[6];
            const double c = joint_coord(type, g, Ja, Jb);
            const double lo = jf[14], hi = jf[15];
            bool use_lo;
            if (isnan(hi)) use_lo = true;
            else if (isnan(lo)) use_lo = false;
            else use_lo = (c - lo) <= (hi - c);
            const float sg = use_lo ? 1.f : -1.f;
            const float gval = (float)(use_lo ? c - lo : hi - c);
            for (int e = 0; e < 6; ++e) {
                Ja[e] *= sg;
                Jb[e] *= sg;
            }
            put_row(row_lim0 + rank, Ja, la, Jb, lb, gval, kRowLimit, 0.f);
        }
        if (fl & kJointDriven) {
            // drive row (Sec. 3 implicit PD, armature, damping; Eq. 2): along
            // the coordinate J_c u+ + R lambda + v* = 0 with
            // K = kp h + kd + d + I_a / dt, R = 1 / (dt K),
            // v* = -(kp (ref - c) + I_a c'- / dt) / K
            int rank = 0;
            for (int q = 0; q < j; ++q) rank += (L.ji(SJTF, q) >> 4) & kJointDriven ? 1 : 0;
            float Ja[6], Jb[6];
            const double c = joint_coord(type, g, Ja, Jb);
            float rate = 0.f;
            for (int e = 0; e < 6; ++e) rate += Ja[e] * L.bf(SBU + e, la);
            if (lb >= 0)
                for (int e = 0; e < 6; ++e) rate += Jb[e] * L.bf(SBU + e, lb);
            const float h = P.integrator == KAMX_MOREAU_JEAN ? 0.5f * P.dt : P.dt;
            const float kp = jf[16], kd = jf[17], ref = jf[18], damp = jf[19], arm = jf[20];
            const float K = kp * h + kd + damp + arm / P.dt;
            const int r = row_drv0 + rank;
            put_row(r, Ja, la, Jb, lb, 0.f, kRowBilateral, 0.f);
            L.rf(SRBIAS, r) = -(float)((double)kp * ((double)ref - c) + (double)arm * (double)rate / (double)P.dt) / K;
            L.rf(SRREG, r) = 1.f / (P.dt * K);
        }
    }
    for (int c = tid; c < nc; c += NT) {
        float p[3], n[3], t1[3], t2[3];
        for (int e = 0; e < 3; ++e) {
            p[e] = L.cf(SCP + e, c);
            n[e] = L.cf(SCN + e, c);
        }
        tangents(n, t1, t2);
        const float *dirs[3] = {n, t1, t2};
        const int la = L.ci(SCA, c), lb = L.ci(SCB, c);
        float arm_a[3], arm_b[3] = {0.f, 0.f, 0.f};
        for (int e = 0; e < 3; ++e) {
            arm_a[e] = p[e] - L.bf(SBQ + e, la);
            if (lb >= 0) arm_b[e] = p[e] - L.bf(SBQ + e, lb);
        }
        for (int e = 0; e < 3; ++e) {
            float Ja[6], Jb[6], cc[3];
            cross(arm_a, dirs[e], cc);
            for (int q = 0; q < 3; ++q) {
                Ja[q] = dirs[e][q];
                Ja[3 + q] = cc[q];
            }
            cross(arm_b, dirs[e], cc);
            for (int q = 0; q < 3; ++q) {
                Jb[q] = -dirs[e][q];
                Jb[3 + q] = -cc[q];
            }
            put_row(rc0p + 4 * c + e, Ja, la, Jb, lb, e == 0 ? L.cf(SCGAP, c) : 0.f,
                    e == 0 ? kRowNormal : kRowTangent, L.cf(SCMU, c));
        }
    }
    __syncthreads();

    // ---- the row of this thread: raw J, bias, kind; compact index
    SpRow R;
    float Jraw[12];
    R.kind = L.ri(SRKIND, tid);
    {
        const int ab = L.rab[tid];
        R.a = (ab & 0xffff) - 1;
        R.b = (ab >> 16) - 1;
    }
    if (R.kind != kRowPad && R.a < 0) R.kind = kRowPad;  // defensive: a row needs a body
    const float bias = L.rf(SRBIAS, tid), mu = L.rf(SRMU, tid), reg = L.rf(SRREG, tid);
    for (int e = 0; e < 12; ++e) Jraw[e] = L.J[e * NT + tid];
    const int qe = (tid - rc0p) & 3;  // lane within a contact quad
    const int ci = tid < row_c0 ? tid : (tid >= rc0p && tid < m_int && qe != 3 ? row_c0 + 3 * ((tid - rc0p) >> 2) + qe : -1);

    // ---- body -> row incidence lists (rows in increasing order), one wave
    //      per body at a time, compacted by ballots
    {
        constexpr int NWAVE = NT / 64;
        const int lane = tid & 63, wave = tid >> 6;
        for (int bb = wave; bb < nb; bb += NWAVE) {
            int cnt = 0;
            for (int r0 = 0; r0 < m_int; r0 += 64) {
                const int r = r0 + lane;
                bool f = false;
                if (r < m_int && L.ri(SRKIND, r) != kRowPad) {
                    const int ab = L.rab[r];
                    f = (ab & 0xffff) - 1 == bb || (ab >> 16) - 1 == bb;
                }
                cnt += __popcll(__ballot(f));
            }
            if (lane == 0) L.inc_off[bb + 1] = cnt;
        }
        __syncthreads();
        if (tid == 0) {
            L.inc_off[0] = 0;
            for (int bb = 0; bb < nb; ++bb) L.inc_off[bb + 1] += L.inc_off[bb];
        }
        __syncthreads();
        for (int bb = wave; bb < nb; bb += NWAVE) {
            int base = L.inc_off[bb];
            for (int r0 = 0; r0 < m_int; r0 += 64) {
                const int r = r0 + lane;
                int side = -1;
                if (r < m_int && L.ri(SRKIND, r) != kRowPad) {
                    const int ab = L.rab[r];
                    if ((ab & 0xffff) - 1 == bb) side = 0;
                    else if ((ab >> 16) - 1 == bb) side = 1;
                }
                const unsigned long long msk = __ballot(side >= 0);
                if (side >= 0) L.inc_list[base + __popcll(msk & ((1ull << lane) - 1ull))] = (r << 1) | side;
                base += __popcll(msk);
            }
        }
    }

    // ---- pre-baked rows: J M^-1/2 per side, the Jacobi scale from the
    //      diagonal D_rr = |J_a M_a^-1/2|^2 + |J_b M_b^-1/2|^2 + R_rr (one
    //      scalar per contact: the trace of its 3x3 block over 3, Sec. 4.1),
    //      J~ = p J M^-1/2, and v~_f = p (J u_f + v*)
    float jh[12];
    float dsum = 0.f;
    if (R.kind != kRowPad) {
        half_inv_mass(L, R.a, Jraw, jh);
        if (R.b >= 0) half_inv_mass(L, R.b, Jraw + 6, jh + 6);
        else
            for (int e = 6; e < 12; ++e) jh[e] = 0.f;
        for (int e = 0; e < 12; ++e) dsum += jh[e] * jh[e];
        dsum += reg;
    } else {
        for (int e = 0; e < 12; ++e) jh[e] = 0.f;
    }
    const float dtr = quad_bc<0>(dsum) + quad_bc<1>(dsum) + quad_bc<2>(dsum);
    float p = 1.f;
    if (R.kind == kRowNormal || R.kind == kRowTangent) {
        const float t = dtr * (1.f / 3.f);
        p = (P.precond && t > 0.f) ? 1.f / sqrtf(t) : 1.f;
    } else if (R.kind != kRowPad) {
        p = (P.precond && dsum > 0.f) ? 1.f / sqrtf(dsum) : 1.f;
    }
    float vf = 0.f;
    if (R.kind != kRowPad) {
        float v = bias;
        for (int e = 0; e < 6; ++e) v += Jraw[e] * L.bf(SBUF + e, R.a);
        if (R.b >= 0)
            for (int e = 0; e < 6; ++e) v += Jraw[6 + e] * L.bf(SBUF + e, R.b);
        vf = p * v;
    }
    for (int e = 0; e < 12; ++e) R.jt[e] = p * jh[e];
    R.preg = p * p * reg;
    __syncthreads();  // raw rows read, incidence lists complete
    for (int e = 0; e < 12; ++e) L.J[e * NT + tid] = R.jt[e];
    // (rho, 1/rho and the shift change only with the adaptive penalty)
    float rho = R.kind == kRowBilateral ? P.rho_bil : (R.kind == kRowPad ? 1.f : P.rho_c);
    float rinv = 1.f / rho;
    const float eta = P.eta;
    float shift = eta + rho;  // diagonal of D~ + diag(eta + rho) beyond D~
    const bool unilateral = R.kind == kRowLimit || R.kind == kRowNormal || R.kind == kRowTangent;

    // ---- warm start (Alg. 1 step 2; Sec. 4.1): y = x = Pi_K(lambda_ws / p),
    //      z = v~(y) + Gamma(v~(y)) on unilateral rows, 0 on bilateral rows;
    //      cold: all zero
    const int wmode = (reset || P.warmstart == KAMX_WARM_LEARNED) ? KAMX_WARM_COLD : P.warmstart;
    float x = 0.f, y = 0.f, z = 0.f, Dx = 0.f;
    if (wmode != KAMX_WARM_COLD) {
        float lw = 0.f;
        if (ci >= 0 && ci < m) {
            if (wmode == KAMX_WARM_EXTERNAL) {
                lw = a.lambda_ext[W.row_base + ci];
            } else if (ci < row_c0) {
                lw = a.lambda[W.row_base + ci];
            } else {
                const int c = (ci - row_c0) / 3, e = (ci - row_c0) - 3 * ((ci - row_c0) / 3);
                const int key = L.ci(SCKEY, c);
                const int nprev = a.ncontacts_out[w];
                for (int q = 0; q < nprev && q < kMaxContacts; ++q)
                    if (a.keys[w * kMaxContacts + q] == key) {
                        lw = a.lambda[W.row_base + row_c0 + 3 * q + e];
                        break;
                    }
            }
        }
        const float ws = (isfinite(lw) && R.kind != kRowPad) ? lw / p : 0.f;
        y = sp_project(R, mu, qe, ws);
        x = y;
        Dx = sp_apply<NT>(L, R, nb, y);
        const float v0 = Dx + vf;
        const float gm = sp_gamma(R, mu, v0);
        z = unilateral ? v0 + gm : 0.f;
    } else {
        __syncthreads();  // J~ visible to the gathers
    }
    float yh = y, zh = z;  // extrapolated iterates
    float yp = y, zp = z;  // iterates of the previous iteration

    // ---- PADMM (Alg. 1 steps 3-10) with the x-update (step 5) by Conjugate
    //      Residual on A = D~ + diag(eta + rho): cr_iters iterations from the
    //      previous x (Sec. 5.1); A x of the previous iterate is known from
    //      the residual evaluation, so the solve starts from
    //      r0 = rhs - A x without a product.
    float a_k = 1.f, c_prev = INFINITY;
    int it = 0, status = 0;
    float rp = 0.f, rd = 0.f, rc = 0.f, rncp = 0.f;
    const int N = P.fixed_iters > 0 ? P.fixed_iters : P.max_iters;
    const int ncr = P.cr_iters > 0 ? P.cr_iters : 1;
    const int n_uni = W.nlim + 3 * nc;  // limit and contact rows: what the adaptive penalty acts on
    bool converged = false;
    for (it = 1; it <= N; ++it) {
        // steps 4-5: s = Gamma(z^), rhs = -v~_f - s + eta x + rho y^ + z^
        const float s = sp_gamma(R, mu, zh);
        const float rhs = R.kind == kRowPad ? 0.f : -vf - s + eta * x + rho * yh + zh;
        float r = rhs - (Dx + shift * x);
        float pc = r;
        float Ap = sp_apply<NT>(L, R, nb, r) + shift * r;
        float sums[4] = {r * Ap, Ap * Ap, 0.f, 0.f};
        sp_sum<NT, 2>(sums, L.red, rbuf);
        float rAr = sums[0], ApAp = sums[1];
        for (int q = 0; q < ncr; ++q) {
            if (!(ApAp > 0.f) || !(rAr > 0.f)) break;  // exact, or no further progress
            const float alpha = rAr / ApAp;
            x += alpha * pc;
            r -= alpha * Ap;
            if (q + 1 == ncr) break;
            const float Ar = sp_apply<NT>(L, R, nb, r) + shift * r;
            float s3[4] = {r * Ar, Ar * Ar, Ar * Ap, 0.f};
            sp_sum<NT, 3>(s3, L.red, rbuf);
            const float beta = s3[0] / rAr;
            rAr = s3[0];
            pc = r + beta * pc;
            Ap = Ar + beta * Ap;
            ApAp = s3[1] + 2.f * beta * s3[2] + beta * beta * ApAp;
        }
        // v~ - v~_f = D~ x for the dual residual and the next right-hand side
        Dx = sp_apply<NT>(L, R, nb, x);
        // steps 6-7
        const float yb = sp_project(R, mu, qe, x - zh * rinv);
        const float zb = zh - rho * (x - yb);
        // step 9: residuals (preconditioned units)
        const float vv = Dx + vf;
        const float gm = sp_gamma(R, mu, vv);
        float lrp = fabsf(x - yb);
        float dres = vv + gm - zb;
        float lrd = fabsf(dres);
        if (dres != dres) lrd = dres;
        // complementarity per unilateral block: y . (v~ + Gamma) over a
        // contact's quad (every lane takes part in the quad sum), y v~ on a
        // limit row
        const bool cont = R.kind == kRowNormal || R.kind == kRowTangent;
        const float qsum = lane_group_sum<4>(cont ? yb * (vv + gm) : 0.f);
        float lrc = R.kind == kRowNormal ? fabsf(qsum) : (R.kind == kRowLimit ? fabsf(yb * vv) : 0.f);
        const float dy = yb - yh, dz = zb - zh;
        float lcc = R.kind == kRowPad ? 0.f : rho * dy * dy + dz * dz * rinv;
        if (R.kind == kRowPad) lrp = lrd = 0.f;
        if (lrp != lrp || lcc != lcc) lrp = NAN;
        sp_max3_sum<NT>(lrp, lrd, lrc, lcc, L.red, rbuf);
        rp = lrp;
        rd = lrd;
        rc = lrc;
        // step 8: Nesterov with adaptive restart
        int restart = 0;
        float beta = 0.f;
        if (P.accel) {
            restart = !(lcc < P.restart_factor * c_prev);
            if (!restart) {
                const float a_next = 0.5f * (1.f + sqrtf(1.f + 4.f * a_k * a_k));
                beta = (a_k - 1.f) / a_next;
                a_k = a_next;
                c_prev = lcc;
            } else {
                a_k = 1.f;
                c_prev = c_prev / P.restart_factor;
            }
        }
        if (!P.accel) {
            yh = yb;
            zh = zb;
        } else if (!restart) {
            yh = yb + beta * (yb - yp);
            zh = zb + beta * (zb - zp);
        } else {
            yh = yp;
            zh = zp;
        }
        yp = yb;
        zp = zb;
        // adaptive penalty (not in the paper: residual balancing) at the
        // checkpoints of a solve that does not exit here; the residuals are
        // the same in every thread, so the decision is uniform
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
            // the limit and contact rows' penalty changes by the factor (the
            // operator is applied matrix-free, so nothing is refactored) and
            // the acceleration restarts at the current (y, z)
            if (unilateral) {
                rho *= adapt_dir == 1 ? 1.f / P.adapt_factor : P.adapt_factor;
                rinv = 1.f / rho;
                shift = eta + rho;
            }
            a_k = 1.f;
            c_prev = INFINITY;
            yh = yp;
            zh = zp;
        }
    }
    if (it > N) it = N;
    if (P.fixed_iters <= 0 && !converged && status == 0) status = KAMX_WORLD_MAXITER;

    // ---- natural-map residual of the NCP at the returned y (Eq. 3); the
    //      product's gather leaves g = J~^T y, which the velocity update uses
    {
        const float Dy = sp_apply<NT>(L, R, nb, yp);
        const float vv = Dy + vf;
        const float gm = sp_gamma(R, mu, vv);
        const float nm = yp - (vv + gm);
        const float o = sp_project(R, mu, qe, nm);
        float lncp = R.kind == kRowPad ? 0.f : fabsf(yp - o);
        float l1 = 0.f, l2 = 0.f, l3 = 0.f;
        sp_max3_sum<NT>(lncp, l1, l2, l3, L.red, rbuf);
        rncp = lncp;
    }

    // ---- outputs: lambda = P y (Alg. 1 step 11) at the compact row index,
    //      statistics, the contact cache
    if (ci >= 0 && ci < W.row_cap) {
        const float lam = p * yp;
        a.lambda[W.row_base + ci] = lam;
        if (a.iterate_out)
            *reinterpret_cast<float4 *>(a.iterate_out + 4 * ((long)W.row_base + ci)) = make_float4(x, yp, zp, p);
    }
    for (int i = m + tid; i < W.row_cap; i += NT) {
        a.lambda[W.row_base + i] = 0.f;
        if (a.iterate_out)
            *reinterpret_cast<float4 *>(a.iterate_out + 4 * ((long)W.row_base + i)) = make_float4(0.f, 0.f, 0.f, 0.f);
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
        ct.body_a = L.ci(SCA, c) + W.b0;
        const int lb = L.ci(SCB, c);
        ct.body_b = lb >= 0 ? lb + W.b0 : -1;
        for (int e = 0; e < 3; ++e) {
            ct.point[e] = L.cf(SCP + e, c);
            ct.normal[e] = L.cf(SCN + e, c);
        }
        ct.gap = L.cf(SCGAP, c);
        ct.mu = L.cf(SCMU, c);
        ct.key = L.ci(SCKEY, c);
        a.contacts_out[w * kMaxContacts + c] = ct;
        a.keys[w * kMaxContacts + c] = ct.key;
    }

    // ---- u+ = u_f + M^-1 J^T lambda = u_f + M^-1/2 (J~^T y) in FP64 from the
    //      gather of the last product, then poses by the exponential map over
    //      the rest of the step (dt, or dt / 2 from the Moreau-Jean half step)
    for (int bb = tid; bb < nb; bb += NT) {
        double gy[6];
        for (int c = 0; c < 6; ++c) gy[c] = L.g[c * kSpBodies + bb];
        const double sm = sqrt((double)L.bf(SBIM, bb));
        double Rm[9], t[3], sv[3];
        for (int c = 0; c < 9; ++c) Rm[c] = L.bf(SBR + c, bb);
        mtv3(Rm, gy + 3, t);
        for (int c = 0; c < 3; ++c) t[c] *= sqrt((double)L.bf(SBII + c, bb));
        mv3(Rm, t, sv);
        float un[6];
        for (int c = 0; c < 3; ++c) {
            un[c] = (float)((double)L.bf(SBUF + c, bb) + gy[c] * sm);
            un[3 + c] = (float)((double)L.bf(SBUF + 3 + c, bb) + sv[c]);
        }
        const int gb = W.b0 + bb;
        for (int e = 0; e < 6; ++e) a.u[6 * gb + e] = un[e];
        double q[7], ud[6], qn[7];
        for (int e = 0; e < 7; ++e) q[e] = L.qd[e * kSpBodies + bb];
        for (int e = 0; e < 6; ++e) ud[e] = un[e];
        advance_pose(q, ud, (P.integrator == KAMX_MOREAU_JEAN ? 0.5 : 1.0) * (double)P.dt, qn);
        for (int e = 0; e < 7; ++e) a.q[7 * gb + e] = (float)qn[e];
    }
    __syncthreads();
}

// A launch advances every world of the bucket by a.nsteps steps, the
// workgroup keeping its world for all of them (as the dense kernel).
template <int NT>
__global__ __launch_bounds__(NT) void sparse_step_kernel(StepArgs a) {
    __shared__ int s_int[8];
    __shared__ StepArgs sa;
    if (threadIdx.x == 0) sa = a;
    __syncthreads();
#pragma clang loop unroll(disable)
    for (int k = 0; k < sa.nsteps; ++k) {
        sparse_step_world<NT>(sa, k, s_int);
        __syncthreads();
    }
}

template <int NT>
static hipError_t launch_sparse(const StepArgs &args, int n, hipStream_t stream) {
    static_assert(NT % 64 == 0 && NT >= 64 && NT <= 1024, "unsupported workgroup size");
    const size_t smem = sizeof(float) * (size_t)sp_smem_floats(NT);
    static bool configured = false;
    if (!configured) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sparse_step_kernel<NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
        configured = true;
    }
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sparse_step_kernel<NT>, dim3(n), dim3(NT), smem, stream, args);
    return hipGetLastError();
}

// Row classes of the matrix-free kernel: one thread per row (contact rows
// in quads), so the class is the workgroup size.
int sparse_row_class(int thread_rows) {
    const int classes[3] = {256, 512, 1024};
    for (int q = 0; q < 3; ++q)
        if (thread_rows <= classes[q]) return classes[q];
    return -1;
}

size_t sparse_smem_bytes(int nt) { return sizeof(float) * (size_t)sp_smem_floats(nt); }

hipError_t launch_sparse_step(const StepArgs &args, int nt, int n, hipStream_t stream) {
    switch (nt) {
    case 256: return launch_sparse<256>(args, n, stream);
    case 512: return launch_sparse<512>(args, n, stream);
    case 1024: return launch_sparse<1024>(args, n, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace kamx
