// Forward kinematics for resets (Sec. 6.3): the poses of every body of a
// world that satisfy all joint constraints -- the passive joints of
// kinematic loops included -- and put the targeted joints at given
// coordinates, found by Gauss-Newton.  One workgroup per world.
//
// Each iteration evaluates, in FP64, F = (the five constraint functions of
// every joint, c_j - target_j for every targeted joint) and its Jacobian J
// over the body twists, and takes the least-change step
//     Delta = -W J^T (J W J^T + mu)^-1 F,   W = M^-1 (the reset body's
//     block zero: it stays where it is),
// moving every body by the exponential map.  The normal matrix is scaled by
// its Jacobi diagonal, regularised by mu = 1e-5 on that unit diagonal (the
// redundant rows of planar loops make J W J^T singular), stored packed in
// LDS in FP32 and factored by a right-looking Cholesky; F and the poses stay
// FP64, so the iteration converges to FP64-level constraint residuals with
// FP32 linear solves.  Runs once per reset, not per step.
#include <math.h>

#include "kamx_geom.h"
#include "kamx_internal.h"

namespace kamx {

namespace {

constexpr int kFkThreads = 256;
constexpr int kFkRows = kMaxRows;
constexpr float kFkMu = 1e-5f;

__host__ __device__ constexpr int fk_tri(int n) { return n * (n + 1) / 2; }

struct FkLds {
    double q[kMaxBodies][7];     // poses
    double F[kFkRows];           // residuals
    double dl[kMaxBodies][6];    // step per body
    float J[kFkRows][12];        // rows: side a, side b
    float W[kFkRows][12];        // M^-1 J^T of both sides
    float p[kFkRows];            // Jacobi scales
    float y[kFkRows];
    float Rm[kMaxBodies][9];     // body rotations
    float red[kFkThreads / 64];
    int ia[kFkRows], ib[kFkRows];
    int trow[kMaxJoints];        // row of a targeted joint, -1
    int flag;
    float A[fk_tri(kFkRows)];    // packed lower triangle, row i at i (i + 1) / 2
};

__device__ inline int tri_index(int i, int j) { return i * (i + 1) / 2 + j; }

// (i, j) with j <= i of the t-th pair of a packed n x n lower triangle
__device__ inline void tri_pair(int t, int &i, int &j) {
    int r = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    i = r;
    j = t - r * (r + 1) / 2;
}

__device__ inline float block_max(float v, float *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float r = red[0];
    for (int k = 1; k < kFkThreads / 64; ++k) r = fmaxf(r, red[k]);
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kFkThreads) void fk_kernel(const WorldInfo *worlds, const int32_t *jint, const float *jf,
                                                        const float *mass, const float *inertia, float *q, float *u,
                                                        const float *targets, int max_iters, float tol,
                                                        int32_t *iters_out, float *resid_out) {
    extern __shared__ float4 smem4[];
    FkLds &S = *reinterpret_cast<FkLds *>(smem4);
    const int tid = threadIdx.x;
    const int w = blockIdx.x;
    const WorldInfo Wd = worlds[w];
    const int nb = Wd.nb, nj = Wd.nj, base = Wd.reset_body;
    for (int t = tid; t < 7 * nb; t += kFkThreads) S.q[t / 7][t % 7] = q[7 * (long)Wd.b0 + t];
    if (tid == 0) {
        int r = 5 * nj;
        for (int j = 0; j < nj; ++j) {
            const float tj = targets[Wd.j0 + j];
            S.trow[j] = isnan(tj) ? -1 : r++;
        }
        S.flag = r;  // row count
    }
    __syncthreads();
    const int m = S.flag;
    if (m > kFkRows) {  // more targets than one world's rows: leave the world alone
        if (tid == 0) {
            if (iters_out) iters_out[w] = 0;
            if (resid_out) resid_out[w] = NAN;
        }
        return;
    }
    int it = 0;
    float fn = INFINITY;
    bool failed = false;
    for (;; ++it) {
        // ---- rows and residuals at the current poses (FP64 geometry)
        for (int j = tid; j < nj; j += kFkThreads) {
            const long gj = Wd.j0 + j;
            const int type = jint[4 * gj], la = jint[4 * gj + 1], lb = jint[4 * gj + 2];
            const float *f = jf + kJointFloats * gj;
            double qb[7];
            for (int k = 0; k < 7; ++k) qb[k] = lb >= 0 ? S.q[lb][k] : 0.0;
            JointGeo g;
            joint_geo_q(S.q[la], qb, lb >= 0, f, g);
            joint_constraints(type, g, [&](int e, const double Ja[6], const double Jb[6], double fv) {
                const int r = 5 * j + e;
                for (int k = 0; k < 6; ++k) {
                    S.J[r][k] = (float)Ja[k];
                    S.J[r][6 + k] = lb >= 0 ? (float)Jb[k] : 0.f;
                }
                S.F[r] = fv;
                S.ia[r] = la;
                S.ib[r] = lb;
            });
            const int rt = S.trow[j];
            if (rt >= 0) {
                float Ja[6], Jb[6];
                const double c = joint_coord(type, g, Ja, Jb);
                for (int k = 0; k < 6; ++k) {
                    S.J[rt][k] = Ja[k];
                    S.J[rt][6 + k] = lb >= 0 ? Jb[k] : 0.f;
                }
                S.F[rt] = c - (double)targets[gj];
                S.ia[rt] = la;
                S.ib[rt] = lb;
            }
        }
        // body rotations for M^-1
        for (int b = tid; b < nb; b += kFkThreads) {
            double R[9], qq[4] = {S.q[b][3], S.q[b][4], S.q[b][5], S.q[b][6]};
            rot_of_quat(qq, R);
            for (int k = 0; k < 9; ++k) S.Rm[b][k] = (float)R[k];
        }
        __syncthreads();
        float lf = 0.f;
        for (int r = tid; r < m; r += kFkThreads) {
            const float a = (float)fabs(S.F[r]);
            lf = (a > lf || a != a) ? a : lf;
        }
        fn = block_max(lf, S.red);
        if (!(fn > tol) || it >= max_iters || failed) break;  // converged, budget spent, or non-finite
        // ---- W = M^-1 J^T per side (body frame: R diag(I^-1) R^T), reset body held
        for (int r = tid; r < m; r += kFkThreads) {
            float dsum = 0.f;
            for (int s = 0; s < 2; ++s) {
                const int b = s ? S.ib[r] : S.ia[r];
                float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (b >= 0 && b != base) {
                    const long gb = Wd.b0 + b;
                    const float im = 1.f / mass[gb];
                    const float *in = S.J[r] + 6 * s;
                    const float *R = S.Rm[b];
                    float t[3], v[3];
                    mtv3(R, in + 3, t);
                    for (int k = 0; k < 3; ++k) t[k] /= inertia[3 * gb + k];
                    mv3(R, t, v);
                    for (int k = 0; k < 3; ++k) {
                        out[k] = in[k] * im;
                        out[3 + k] = v[k];
                    }
                }
                for (int k = 0; k < 6; ++k) {
                    S.W[r][6 * s + k] = out[k];
                    dsum += S.J[r][6 * s + k] * out[k];
                }
            }
            S.p[r] = dsum > 0.f ? 1.f / sqrtf(dsum) : 1.f;
        }
        __syncthreads();
        // ---- scaled normal matrix P J W J^T P + mu (rows sharing a body only)
        for (int t = tid; t < fk_tri(m); t += kFkThreads) {
            int i, j;
            tri_pair(t, i, j);
            float acc = 0.f;
            const int bi[2] = {S.ia[i], S.ib[i]}, bj[2] = {S.ia[j], S.ib[j]};
            for (int s = 0; s < 2; ++s)
                for (int v = 0; v < 2; ++v)
                    if (bi[s] >= 0 && bi[s] == bj[v])
                        for (int k = 0; k < 6; ++k) acc += S.J[i][6 * s + k] * S.W[j][6 * v + k];
            acc *= S.p[i] * S.p[j];
            if (i == j) acc += kFkMu;
            S.A[t] = acc;
        }
        if (tid == 0) S.flag = 0;
        __syncthreads();
        // ---- Cholesky, right-looking by columns
        for (int k = 0; k < m; ++k) {
            if (tid == 0) {
                const float d = S.A[tri_index(k, k)];
                if (!(d > 0.f)) S.flag = 1;
                S.A[tri_index(k, k)] = d > 0.f ? sqrtf(d) : 1.f;
            }
            __syncthreads();
            const float lkk = S.A[tri_index(k, k)];
            for (int i = k + 1 + tid; i < m; i += kFkThreads) S.A[tri_index(i, k)] /= lkk;
            __syncthreads();
            const int n = m - k - 1;
            for (int t = tid; t < fk_tri(n); t += kFkThreads) {
                int i, j;
                tri_pair(t, i, j);
                i += k + 1;
                j += k + 1;
                S.A[tri_index(i, j)] -= S.A[tri_index(i, k)] * S.A[tri_index(j, k)];
            }
            __syncthreads();
        }
        if (S.flag) {
            failed = true;
            continue;  // reported as a non-finite residual below
        }
        // ---- solve (P A P) y~ = P F, then y = P y~
        for (int r = tid; r < m; r += kFkThreads) S.y[r] = S.p[r] * (float)S.F[r];
        __syncthreads();
        for (int k = 0; k < m; ++k) {
            if (tid == 0) S.y[k] /= S.A[tri_index(k, k)];
            __syncthreads();
            const float yk = S.y[k];
            for (int i = k + 1 + tid; i < m; i += kFkThreads) S.y[i] -= S.A[tri_index(i, k)] * yk;
            __syncthreads();
        }
        for (int k = m - 1; k >= 0; --k) {
            if (tid == 0) S.y[k] /= S.A[tri_index(k, k)];
            __syncthreads();
            const float yk = S.y[k];
            for (int i = tid; i < k; i += kFkThreads) S.y[i] -= S.A[tri_index(k, i)] * yk;
            __syncthreads();
        }
        for (int r = tid; r < m; r += kFkThreads) S.y[r] *= S.p[r];
        __syncthreads();
        // ---- Delta = -W J^T y per body component (rows in order), FP64
        for (int t = tid; t < 6 * nb; t += kFkThreads) {
            const int b = t / 6, c = t - 6 * (t / 6);
            double acc = 0.0;
            for (int r = 0; r < m; ++r) {
                if (S.ia[r] == b) acc += (double)S.W[r][c] * (double)S.y[r];
                if (S.ib[r] == b) acc += (double)S.W[r][6 + c] * (double)S.y[r];
            }
            S.dl[b][c] = -acc;
        }
        __syncthreads();
        // ---- move every body: r += Delta_v, R <- exp(Delta_w) R
        for (int b = tid; b < nb; b += kFkThreads) {
            const double *d = S.dl[b];
            for (int k = 0; k < 3; ++k) S.q[b][k] += d[k];
            const double wn = sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
            if (wn > 0.0) {
                const double sh = sin(0.5 * wn) / wn;
                const double dq[4] = {d[3] * sh, d[4] * sh, d[5] * sh, cos(0.5 * wn)};
                double qo[4] = {S.q[b][3], S.q[b][4], S.q[b][5], S.q[b][6]}, qn[4];
                qprod(dq, qo, qn);
                const double nn = 1.0 / sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
                for (int k = 0; k < 4; ++k) S.q[b][3 + k] = qn[k] * nn;
            }
        }
        __syncthreads();
    }
    // poses out (FP32), twists zero
    for (int t = tid; t < 7 * nb; t += kFkThreads) q[7 * (long)Wd.b0 + t] = (float)S.q[t / 7][t % 7];
    for (int t = tid; t < 6 * nb; t += kFkThreads) u[6 * (long)Wd.b0 + t] = 0.f;
    if (tid == 0) {
        if (iters_out) iters_out[w] = it;
        if (resid_out) resid_out[w] = failed ? NAN : fn;
    }
}

}  // namespace

size_t fk_smem_bytes() { return sizeof(FkLds); }

hipError_t launch_fk(const WorldInfo *worlds, int n_worlds, const int32_t *jint, const float *jf, const float *mass,
                     const float *inertia, float *q, float *u, const float *targets, int max_iters, float tol,
                     int32_t *iters, float *resid, hipStream_t stream) {
    if (n_worlds <= 0) return hipSuccess;
    static bool configured = false;
    const size_t bytes = sizeof(FkLds);
    if (!configured) {
        hipError_t e = hipFuncSetAttribute((const void *)fk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)bytes);
        if (e != hipSuccess) return e;
        configured = true;
    }
    hipLaunchKernelGGL(fk_kernel, dim3(n_worlds), dim3(kFkThreads), bytes, stream, worlds, jint, jf, mass, inertia, q,
                       u, targets, max_iters, tol, iters, resid);
    return hipGetLastError();
}

}  // namespace kamx
