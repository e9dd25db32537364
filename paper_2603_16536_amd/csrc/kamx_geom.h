// Small device geometry shared by the step kernel and the kinematics
// kernel: rotations and vector products, and the joint geometry of Sec. 3
// (anchors, frames, the joint coordinate and its Jacobian) evaluated in FP64.
#pragma once

#include <math.h>

#include "kamx_internal.h"

namespace kamx {

// ---------------------------------------------------------------------------
// small device math
// ---------------------------------------------------------------------------

template <typename T>
__device__ inline void rot_of_quat(const T q[4], T R[9]) {
    T x = q[0], y = q[1], z = q[2], w = q[3];
    R[0] = T(1) - T(2) * (y * y + z * z);
    R[1] = T(2) * (x * y - z * w);
    R[2] = T(2) * (x * z + y * w);
    R[3] = T(2) * (x * y + z * w);
    R[4] = T(1) - T(2) * (x * x + z * z);
    R[5] = T(2) * (y * z - x * w);
    R[6] = T(2) * (x * z - y * w);
    R[7] = T(2) * (y * z + x * w);
    R[8] = T(1) - T(2) * (x * x + y * y);
}

template <typename T>
__device__ inline void qprod(const T p[4], const T q[4], T r[4]) {
    r[0] = p[3] * q[0] + p[0] * q[3] + p[1] * q[2] - p[2] * q[1];
    r[1] = p[3] * q[1] - p[0] * q[2] + p[1] * q[3] + p[2] * q[0];
    r[2] = p[3] * q[2] + p[0] * q[1] - p[1] * q[0] + p[2] * q[3];
    r[3] = p[3] * q[3] - p[0] * q[0] - p[1] * q[1] - p[2] * q[2];
}

template <typename T>
__device__ inline void cross(const T a[3], const T b[3], T c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

template <typename T>
__device__ inline T dot3(const T a[3], const T b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

template <typename T>
__device__ inline void mv3(const T R[9], const T v[3], T o[3]) {
    o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}

template <typename T>
__device__ inline void mtv3(const T R[9], const T v[3], T o[3]) {
    o[0] = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
    o[1] = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
    o[2] = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
}

// Joint geometry: anchors, lever arms and frame rotations of both sides.
// Evaluated in FP64: the Baumgarte bias multiplies the position-level
// constraint value by beta / dt, so FP32 rounding of near-cancelling anchor
// offsets and near-orthogonal axis products (about 1e-7 absolute) would
// become velocity errors of order 1e-5.  J and everything downstream stay
// FP32.
struct JointGeo {
    double pa[3], pb[3], ra[3], rb[3], Ra[9], Rb[9];
};

// From the poses (position, quaternion) of side a and side b (has_b = false:
// the world; qb7 is then not read) and the joint's frames jf (frame a 7,
// frame b 7).
__device__ inline void joint_geo_q(const double qa[7], const double qb7[7], bool has_b, const float *jf,
                                   JointGeo &g) {
    double Rbody[9], t[3], qq[4], qb[4], fr[4], c[3];
    for (int k = 0; k < 4; ++k) qb[k] = qa[3 + k];
    rot_of_quat(qb, Rbody);
    for (int k = 0; k < 3; ++k) c[k] = jf[k];
    mv3(Rbody, c, t);
    for (int k = 0; k < 3; ++k) {
        g.ra[k] = qa[k];
        g.pa[k] = g.ra[k] + t[k];
    }
    for (int k = 0; k < 4; ++k) fr[k] = jf[3 + k];
    qprod(qb, fr, qq);
    rot_of_quat(qq, g.Ra);
    for (int k = 0; k < 4; ++k) fr[k] = jf[10 + k];
    if (has_b) {
        for (int k = 0; k < 4; ++k) qb[k] = qb7[3 + k];
        rot_of_quat(qb, Rbody);
        for (int k = 0; k < 3; ++k) c[k] = jf[7 + k];
        mv3(Rbody, c, t);
        for (int k = 0; k < 3; ++k) {
            g.rb[k] = qb7[k];
            g.pb[k] = g.rb[k] + t[k];
        }
        qprod(qb, fr, qq);
        rot_of_quat(qq, g.Rb);
    } else {
        for (int k = 0; k < 3; ++k) {
            g.rb[k] = 0.0;
            g.pb[k] = jf[7 + k];
        }
        rot_of_quat(fr, g.Rb);
    }
}

__device__ inline void col(const double R[9], int k, double c[3]) {
    c[0] = R[k];
    c[1] = R[3 + k];
    c[2] = R[6 + k];
}

// Joint coordinate and its Jacobian (6-vectors for sides a and b).
__device__ inline double joint_coord(int type, const JointGeo &g, float Ja[6], float Jb[6]) {
    double Xb[3], Yb[3], Zb[3], Ya[3];
    col(g.Rb, 0, Xb);
    col(g.Rb, 1, Yb);
    col(g.Rb, 2, Zb);
    col(g.Ra, 1, Ya);
    if (type == KAMX_REVOLUTE) {
        for (int k = 0; k < 3; ++k) {
            Ja[k] = 0.f;
            Jb[k] = 0.f;
            Ja[3 + k] = (float)Xb[k];
            Jb[3 + k] = (float)-Xb[k];
        }
        return atan2(dot3(Ya, Zb), dot3(Ya, Yb));
    }
    double d[3], la[3], lb[3], c[3];
    for (int k = 0; k < 3; ++k) {
        d[k] = g.pa[k] - g.pb[k];
        la[k] = g.pa[k] - g.ra[k];
        lb[k] = g.pa[k] - g.rb[k];
    }
    cross(la, Xb, c);
    for (int k = 0; k < 3; ++k) {
        Ja[k] = (float)Xb[k];
        Ja[3 + k] = (float)c[k];
    }
    cross(lb, Xb, c);
    for (int k = 0; k < 3; ++k) {
        Jb[k] = (float)-Xb[k];
        Jb[3 + k] = (float)-c[k];
    }
    return dot3(d, Xb);
}

// The five constraint functions of a joint (Sec. 3) and their Jacobians in
// FP64: revolute = anchor coincidence p_a - p_b (3) and axis alignment
// X_a.Y_b, X_a.Z_b (2); prismatic = anchor offset (p_a - p_b).Y_b, .Z_b (2)
// and orientation lock X_a.Y_b, X_a.Z_b, Y_a.Z_b (3).  emit(e, Ja, Jb, f)
// receives constraint e.
template <typename Emit>
__device__ inline void joint_constraints(int type, const JointGeo &g, Emit &&emit) {
    double Xa[3], Ya[3], Yb[3], Zb[3];
    col(g.Ra, 0, Xa);
    col(g.Ra, 1, Ya);
    col(g.Rb, 1, Yb);
    col(g.Rb, 2, Zb);
    double arm_a[3], arm_b[3], d[3];
    for (int k = 0; k < 3; ++k) {
        arm_a[k] = g.pa[k] - g.ra[k];
        arm_b[k] = g.pb[k] - g.rb[k];
        d[k] = g.pa[k] - g.pb[k];
    }
    double Ja[6], Jb[6], c[3];
    if (type == KAMX_REVOLUTE) {
        for (int e = 0; e < 3; ++e) {
            double ek[3] = {0.0, 0.0, 0.0};
            ek[e] = 1.0;
            cross(arm_a, ek, c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = ek[k];
                Ja[3 + k] = c[k];
            }
            cross(arm_b, ek, c);
            for (int k = 0; k < 3; ++k) {
                Jb[k] = -ek[k];
                Jb[3 + k] = -c[k];
            }
            emit(e, Ja, Jb, d[e]);
        }
        const double *T[2] = {Yb, Zb};
        for (int e = 0; e < 2; ++e) {
            cross(Xa, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = 0.0;
                Ja[3 + k] = c[k];
                Jb[k] = 0.0;
                Jb[3 + k] = -c[k];
            }
            emit(3 + e, Ja, Jb, dot3(Xa, T[e]));
        }
    } else {
        double lever_b[3];
        for (int k = 0; k < 3; ++k) lever_b[k] = g.pa[k] - g.rb[k];
        const double *T[2] = {Yb, Zb};
        for (int e = 0; e < 2; ++e) {
            cross(arm_a, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = T[e][k];
                Ja[3 + k] = c[k];
            }
            cross(lever_b, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Jb[k] = -T[e][k];
                Jb[3 + k] = -c[k];
            }
            emit(e, Ja, Jb, dot3(d, T[e]));
        }
        const double *U[3] = {Xa, Xa, Ya};
        const double *V[3] = {Yb, Zb, Zb};
        for (int e = 0; e < 3; ++e) {
            cross(U[e], V[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = 0.0;
                Ja[3 + k] = c[k];
                Jb[k] = 0.0;
                Jb[3 + k] = -c[k];
            }
            emit(2 + e, Ja, Jb, dot3(U[e], V[e]));
        }
    }
}

}  // namespace kamx
