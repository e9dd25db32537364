/*
 * kamx_oracle.c -- plain FP64 CPU reference of one constrained
 * forward-dynamics time step for a batch of maximal-coordinate worlds.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle against which the HIP
 * library is checked.  Only the tests, the smoke check and the CPU baseline
 * leg of the benchmark load it; the library never does.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * It follows "Kamino: GPU-based Massively Parallel Simulation of Multi-Body
 * Systems with Challenging Topologies" (Tsounis et al., 2026):
 *   Sec. 3, Eq. 1     block-diagonal mass matrix, Newton-Euler forces h
 *   Sec. 3            joint / limit / contact constraints, Baumgarte bias,
 *                     semi-implicit Euler with the SO(3) exponential map
 *   Sec. 4, Eq. 3-4   dual problem, Delassus D and free velocity v_f
 *   Sec. 4, Alg. 1    Proximal-ADMM (PADMM)
 *   Sec. 4.1          Nesterov acceleration with restart, Jacobi
 *                     preconditioning, three infinity-norm residuals
 *   Sec. 3, Eq. 2     joint-space drives (implicit PD, armature, viscous
 *                     damping) as regularised rows: R on the diagonal of
 *                     D, their targets in v*
 *   Sec. 3            the Moreau-Jean midpoint variant of the time step
 *   Sec. 6.3          forward kinematics by Gauss-Newton (consistent poses
 *                     from target joint coordinates, for resets)
 *   Sec. 5.1          the iterative linear solve of Alg. 1 step 5: Conjugate
 *                     Residual with a fixed budget, warm-started at the
 *                     previous iterate, on the Delassus operator
 * Where the paper is silent the readings are stated next to the code that
 * uses them.  Everything is written for clarity: dense J (m x 6 n_b), dense
 * D = J M^-1 J^T, a textbook Cholesky and two triangular solves per
 * iteration.  No blocking, no fusion.
 *
 * Conventions: quaternions (x, y, z, w); twists (v, w) with w in the world
 * frame; a joint couples body a (a real body) and body b (-1 = world); the
 * joint axis is the x axis of each side's frame; a contact normal points
 * from body b to body a and a positive normal impulse separates them.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_REVOLUTE 0
#define ORC_PRISMATIC 1

/* row kinds */
#define ORC_ROW_BILATERAL 0
#define ORC_ROW_LIMIT 1
#define ORC_ROW_NORMAL 2
#define ORC_ROW_TANGENT 3

/* per-world status bits */
#define ORC_OK 0
#define ORC_MAXITER 1
#define ORC_NONFINITE 2
#define ORC_FACTOR_FAIL 4

typedef struct {
    double dt;
    double gravity[3];
    double eta;            /* proximal parameter                          */
    double rho_bil;        /* ADMM penalty on bilateral rows              */
    double rho_c;          /* ADMM penalty on limit and contact rows      */
    double eps;            /* tolerance of the three residuals            */
    int32_t max_iters;     /* iteration cap                                */
    int32_t fixed_iters;   /* >0: exactly this many iterations, no exit    */
    int32_t accel;         /* Nesterov acceleration with restart           */
    double restart_factor; /* gamma of the restart test                    */
    int32_t precond;       /* Jacobi preconditioning                       */
    double baumgarte;      /* beta                                         */
    int32_t warmstart;     /* 0 cold, 1 from lambda_ws                     */
    int32_t replay;        /* 1: restart decisions read from restart_log   */
    int32_t log_stride;    /* bytes per world in restart_log               */
    int32_t integrator;    /* 0 semi-implicit Euler, 1 Moreau-Jean midpoint */
    int32_t cr_iters;      /* 0: Cholesky; > 0: that many Conjugate Residual
                              iterations per x-update (Sec. 5.1)          */
    double adapt_ratio;    /* > 0: adaptive penalty on limit and contact
                              rows (residual balancing, see the solver)   */
    double adapt_factor;   /* factor of one penalty change                 */
    int32_t adapt_first;   /* first checkpoint iteration (then doubling)   */
} orc_params;

typedef struct {
    int32_t n_worlds;
    int32_t n_bodies;
    const int32_t *body_world;   /* [nb], sorted                       */
    const double *mass;          /* [nb]                               */
    const double *inertia;       /* [nb*3] principal, body frame        */
    int32_t n_joints;
    const int32_t *joint_type;   /* [nj]                               */
    const int32_t *joint_world;  /* [nj], sorted                       */
    const int32_t *joint_body;   /* [nj*2] global body ids, b may be -1 */
    const double *joint_frame;   /* [nj*14] frame a (p, q), frame b    */
    const double *joint_limit;   /* [nj*2] lo, hi (NaN = none)         */
    int32_t n_contacts;
    const int32_t *contact_world;   /* [nc], sorted                    */
    const int32_t *contact_body;    /* [nc*2]                          */
    const double *contact_point;    /* [nc*3] world                    */
    const double *contact_normal;   /* [nc*3] unit, from b to a         */
    const double *contact_gap;      /* [nc]                            */
    const double *contact_mu;       /* [nc]                            */
    const double *joint_drive;      /* [nj*5] kp, kd, damping, armature,
                                       ref of implicit drives, or NULL   */
} orc_batch;

typedef struct {
    const double *q;            /* [nb*7] poses before the step          */
    const double *u;            /* [nb*6] twists before the step         */
    const double *joint_torque; /* [nj] generalized joint force, or NULL */
    const double *lambda_ws;    /* [rows] warm start (physical), or NULL */
    double *q_out;              /* [nb*7]                                */
    double *u_out;              /* [nb*6]                                */
    double *lambda;             /* [rows] impulses (physical units)      */
    double *lambda_tilde;       /* [rows] preconditioned y, or NULL      */
    int64_t *row_offset;        /* [nw+1]                                */
    int32_t *iters;             /* [nw]                                  */
    double *resid;              /* [nw*4]: r_p, r_d, r_c, r_ncp          */
    int32_t *status;            /* [nw]                                  */
    uint8_t *restart_log;       /* [nw*log_stride] or NULL               */
} orc_io;

/* ------------------------------------------------------------------------ */
/* small vector and rotation helpers                                         */
/* ------------------------------------------------------------------------ */

static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* rotation matrix (row-major) of a unit quaternion (x, y, z, w) */
static void quat_to_rot(const double *q, double *R) {
    double x = q[0], y = q[1], z = q[2], w = q[3];
    R[0] = 1 - 2 * (y * y + z * z);
    R[1] = 2 * (x * y - z * w);
    R[2] = 2 * (x * z + y * w);
    R[3] = 2 * (x * y + z * w);
    R[4] = 1 - 2 * (x * x + z * z);
    R[5] = 2 * (y * z - x * w);
    R[6] = 2 * (x * z - y * w);
    R[7] = 2 * (y * z + x * w);
    R[8] = 1 - 2 * (x * x + y * y);
}

static void quat_mul(const double *p, const double *q, double *r) {
    r[0] = p[3] * q[0] + p[0] * q[3] + p[1] * q[2] - p[2] * q[1];
    r[1] = p[3] * q[1] - p[0] * q[2] + p[1] * q[3] + p[2] * q[0];
    r[2] = p[3] * q[2] + p[0] * q[1] - p[1] * q[0] + p[2] * q[3];
    r[3] = p[3] * q[3] - p[0] * q[0] - p[1] * q[1] - p[2] * q[2];
}

static void mat_vec3(const double *R, const double *v, double *o) {
    o[0] = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
    o[1] = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
    o[2] = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
}

/* world-frame rotation of a frame with body pose q_body and local quat q_loc */
static void frame_rot(const double *q_body, const double *q_loc, double *R) {
    double qq[4];
    if (q_body) {
        quat_mul(q_body, q_loc, qq);
        quat_to_rot(qq, R);
    } else {
        quat_to_rot(q_loc, R);
    }
}

/* column k of a row-major 3x3 */
static void col3(const double *R, int k, double *c) {
    c[0] = R[k];
    c[1] = R[3 + k];
    c[2] = R[6 + k];
}

/* Orthonormal tangents t1, t2 completing a unit normal n (Duff, Burgess,
 * Christensen, Hery, Kensler, Liani, Villemin, "Building an Orthonormal
 * Basis, Revisited", JCGT 6(1), 2017). */
static void tangent_basis(const double *n, double *t1, double *t2) {
    double sgn = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sgn + n[2]);
    double b = n[0] * n[1] * a;
    t1[0] = 1.0 + sgn * n[0] * n[0] * a;
    t1[1] = sgn * b;
    t1[2] = -sgn * n[0];
    t2[0] = b;
    t2[1] = sgn + n[1] * n[1] * a;
    t2[2] = -n[1];
}

/* ------------------------------------------------------------------------ */
/* one world's assembled problem                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int nb, m, b0;          /* bodies, rows, first global body */
    double *J;              /* [m][6 nb]                       */
    double *f;              /* [m] position-level value        */
    double *vstar;          /* [m] bias                        */
    int *kind;              /* [m]                             */
    double *mu;             /* [m] friction (contact rows)     */
    double *Minv;           /* [nb][6][6]                      */
    double *uf;             /* [6 nb] free velocity of bodies  */
    double *Rreg;           /* [m] diagonal regularisation R   */
} world_sys;

static int joint_rows(int type) {
    (void)type;
    return 5; /* revolute and prismatic each lock 5 DoF */
}

static int has_limit(const double *lim) { return !isnan(lim[0]) || !isnan(lim[1]); }

/* a joint has a drive row when any of its drive gains is nonzero */
static int has_drive(const orc_batch *B, int j) {
    if (!B->joint_drive) return 0;
    const double *d = B->joint_drive + 5 * (size_t)j;
    return d[0] != 0.0 || d[1] != 0.0 || d[2] != 0.0 || d[3] != 0.0;
}

/* the world-local body index of global body b (or -1 for the world) */
static int local_body(int b, int b0) { return b < 0 ? -1 : b - b0; }

/* Write row r of J for a two-body row: J_a, J_b as 6-vectors. */
static void put_row(world_sys *S, int r, int la, const double *Ja, int lb, const double *Jb) {
    double *row = S->J + (size_t)r * 6 * S->nb;
    if (la >= 0)
        for (int k = 0; k < 6; ++k) row[6 * la + k] += Ja[k];
    if (lb >= 0)
        for (int k = 0; k < 6; ++k) row[6 * lb + k] += Jb[k];
}

typedef struct {
    double pa[3], pb[3];      /* anchor points, world              */
    double ra[3], rb[3];      /* body origins (0 for the world)    */
    double Ra[9], Rb[9];      /* frame rotations, world            */
} joint_geo;

static void joint_geometry(const orc_batch *B, const double *q, int j, joint_geo *g) {
    const double *fr = B->joint_frame + 14 * (size_t)j;
    int a = B->joint_body[2 * j], b = B->joint_body[2 * j + 1];
    const double *qa = q + 7 * (size_t)a;
    double Rba[9], tmp[3];
    quat_to_rot(qa + 3, Rba);
    mat_vec3(Rba, fr, tmp);
    for (int k = 0; k < 3; ++k) {
        g->ra[k] = qa[k];
        g->pa[k] = qa[k] + tmp[k];
    }
    frame_rot(qa + 3, fr + 3, g->Ra);
    if (b >= 0) {
        const double *qb = q + 7 * (size_t)b;
        double Rbb[9];
        quat_to_rot(qb + 3, Rbb);
        mat_vec3(Rbb, fr + 7, tmp);
        for (int k = 0; k < 3; ++k) {
            g->rb[k] = qb[k];
            g->pb[k] = qb[k] + tmp[k];
        }
        frame_rot(qb + 3, fr + 10, g->Rb);
    } else {
        for (int k = 0; k < 3; ++k) {
            g->rb[k] = 0.0;
            g->pb[k] = fr[7 + k];
        }
        frame_rot(NULL, fr + 10, g->Rb);
    }
}

/* Joint coordinate (revolute angle of A about the axis relative to B, or
 * prismatic extension of A's anchor along B's axis) and its Jacobian. */
static double joint_coordinate(const orc_batch *B, const double *q, int j, double *Ja, double *Jb) {
    joint_geo g;
    joint_geometry(B, q, j, &g);
    double Xb[3], Yb[3], Zb[3], Ya[3];
    col3(g.Rb, 0, Xb);
    col3(g.Rb, 1, Yb);
    col3(g.Rb, 2, Zb);
    col3(g.Ra, 1, Ya);
    if (B->joint_type[j] == ORC_REVOLUTE) {
        for (int k = 0; k < 3; ++k) {
            Ja[k] = 0.0;
            Jb[k] = 0.0;
            Ja[3 + k] = Xb[k];
            Jb[3 + k] = -Xb[k];
        }
        return atan2(dot3(Ya, Zb), dot3(Ya, Yb));
    } else {
        double d[3], la[3], lb[3], c[3];
        for (int k = 0; k < 3; ++k) {
            d[k] = g.pa[k] - g.pb[k];
            la[k] = g.pa[k] - g.ra[k];
            lb[k] = g.pa[k] - g.rb[k];
        }
        cross3(la, Xb, c);
        for (int k = 0; k < 3; ++k) {
            Ja[k] = Xb[k];
            Ja[3 + k] = c[k];
        }
        cross3(lb, Xb, c);
        for (int k = 0; k < 3; ++k) {
            Jb[k] = -Xb[k];
            Jb[3 + k] = -c[k];
        }
        return dot3(d, Xb);
    }
}

/* Rows of joint j starting at row r0: Sec. 3 bilateral constraints
 * f(q) = 0.  Revolute: anchor coincidence (3) + axis alignment (2).
 * Prismatic: anchor offset normal to the axis (2) + full orientation
 * lock (3).  J is the exact time derivative of f along the twists. */
static void assemble_joint(const orc_batch *B, const double *q, int j, world_sys *S, int r0) {
    joint_geo g;
    joint_geometry(B, q, j, &g);
    int a = B->joint_body[2 * j], b = B->joint_body[2 * j + 1];
    int la = local_body(a, S->b0), lb = local_body(b, S->b0);
    double Xa[3], Ya[3], Yb[3], Zb[3];
    col3(g.Ra, 0, Xa);
    col3(g.Ra, 1, Ya);
    col3(g.Rb, 1, Yb);
    col3(g.Rb, 2, Zb);
    double arm_a[3], arm_b[3], d[3];
    for (int k = 0; k < 3; ++k) {
        arm_a[k] = g.pa[k] - g.ra[k];
        arm_b[k] = g.pb[k] - g.rb[k];
        d[k] = g.pa[k] - g.pb[k];
    }
    double Ja[6], Jb[6], c[3];
    if (B->joint_type[j] == ORC_REVOLUTE) {
        for (int e = 0; e < 3; ++e) {
            double ek[3] = {0, 0, 0};
            ek[e] = 1.0;
            cross3(arm_a, ek, c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = ek[k];
                Ja[3 + k] = c[k];
            }
            cross3(arm_b, ek, c);
            for (int k = 0; k < 3; ++k) {
                Jb[k] = -ek[k];
                Jb[3 + k] = -c[k];
            }
            put_row(S, r0 + e, la, Ja, lb, Jb);
            S->f[r0 + e] = d[e];
            S->kind[r0 + e] = ORC_ROW_BILATERAL;
        }
        const double *T[2] = {Yb, Zb};
        for (int e = 0; e < 2; ++e) {
            cross3(Xa, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = 0.0;
                Ja[3 + k] = c[k];
                Jb[k] = 0.0;
                Jb[3 + k] = -c[k];
            }
            put_row(S, r0 + 3 + e, la, Ja, lb, Jb);
            S->f[r0 + 3 + e] = dot3(Xa, T[e]);
            S->kind[r0 + 3 + e] = ORC_ROW_BILATERAL;
        }
    } else {
        /* anchor offset along B's perpendicular axes */
        double lever_b[3];
        for (int k = 0; k < 3; ++k) lever_b[k] = g.pa[k] - g.rb[k];
        const double *T[2] = {Yb, Zb};
        for (int e = 0; e < 2; ++e) {
            cross3(arm_a, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = T[e][k];
                Ja[3 + k] = c[k];
            }
            cross3(lever_b, T[e], c);
            for (int k = 0; k < 3; ++k) {
                Jb[k] = -T[e][k];
                Jb[3 + k] = -c[k];
            }
            put_row(S, r0 + e, la, Ja, lb, Jb);
            S->f[r0 + e] = dot3(d, T[e]);
            S->kind[r0 + e] = ORC_ROW_BILATERAL;
        }
        /* orientation lock: Xa.Yb, Xa.Zb, Ya.Zb */
        const double *U[3] = {Xa, Xa, Ya};
        const double *V[3] = {Yb, Zb, Zb};
        for (int e = 0; e < 3; ++e) {
            cross3(U[e], V[e], c);
            for (int k = 0; k < 3; ++k) {
                Ja[k] = 0.0;
                Ja[3 + k] = c[k];
                Jb[k] = 0.0;
                Jb[3 + k] = -c[k];
            }
            put_row(S, r0 + 2 + e, la, Ja, lb, Jb);
            S->f[r0 + 2 + e] = dot3(U[e], V[e]);
            S->kind[r0 + 2 + e] = ORC_ROW_BILATERAL;
        }
    }
}

/* Sec. 3 unilateral limit 0 <= lambda _|_ g(q) >= 0 on the joint
 * coordinate.  One row per limited joint, against the nearer bound. */
static void assemble_limit(const orc_batch *B, const double *q, int j, world_sys *S, int r) {
    double Ja[6], Jb[6];
    double c = joint_coordinate(B, q, j, Ja, Jb);
    const double *lim = B->joint_limit + 2 * (size_t)j;
    double sgn, gval;
    int use_lo;
    if (isnan(lim[1])) use_lo = 1;
    else if (isnan(lim[0])) use_lo = 0;
    else use_lo = (c - lim[0]) <= (lim[1] - c);
    if (use_lo) {
        sgn = 1.0;
        gval = c - lim[0];
    } else {
        sgn = -1.0;
        gval = lim[1] - c;
    }
    for (int k = 0; k < 6; ++k) {
        Ja[k] *= sgn;
        Jb[k] *= sgn;
    }
    int a = B->joint_body[2 * j], b = B->joint_body[2 * j + 1];
    put_row(S, r, local_body(a, S->b0), Ja, local_body(b, S->b0), Jb);
    S->f[r] = gval;
    S->kind[r] = ORC_ROW_LIMIT;
}

/* Sec. 3 frictional contact: rows (n, t1, t2) of the relative velocity of
 * body a's material point w.r.t. body b's at the contact point. */
static void assemble_contact(const orc_batch *B, const double *q, int c, world_sys *S, int r) {
    const double *p = B->contact_point + 3 * (size_t)c;
    const double *n = B->contact_normal + 3 * (size_t)c;
    double t1[3], t2[3];
    tangent_basis(n, t1, t2);
    const double *dirs[3] = {n, t1, t2};
    int a = B->contact_body[2 * c], b = B->contact_body[2 * c + 1];
    double arm_a[3] = {0, 0, 0}, arm_b[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        arm_a[k] = p[k] - q[7 * (size_t)a + k];
        if (b >= 0) arm_b[k] = p[k] - q[7 * (size_t)b + k];
    }
    for (int e = 0; e < 3; ++e) {
        double Ja[6], Jb[6], cc[3];
        cross3(arm_a, dirs[e], cc);
        for (int k = 0; k < 3; ++k) {
            Ja[k] = dirs[e][k];
            Ja[3 + k] = cc[k];
        }
        cross3(arm_b, dirs[e], cc);
        for (int k = 0; k < 3; ++k) {
            Jb[k] = -dirs[e][k];
            Jb[3 + k] = -cc[k];
        }
        put_row(S, r + e, local_body(a, S->b0), Ja, local_body(b, S->b0), Jb);
        S->f[r + e] = e == 0 ? B->contact_gap[c] : 0.0;
        S->kind[r + e] = e == 0 ? ORC_ROW_NORMAL : ORC_ROW_TANGENT;
        S->mu[r + e] = B->contact_mu[c];
    }
}

/* world ranges */
typedef struct {
    int b0, b1, j0, j1, c0, c1;
} world_range;

static void find_range(const int32_t *ids, int n, int w, int *lo, int *hi) {
    int i = 0;
    while (i < n && ids[i] < w) ++i;
    *lo = i;
    while (i < n && ids[i] == w) ++i;
    *hi = i;
}

static world_range get_range(const orc_batch *B, int w) {
    world_range R;
    find_range(B->body_world, B->n_bodies, w, &R.b0, &R.b1);
    find_range(B->joint_world, B->n_joints, w, &R.j0, &R.j1);
    find_range(B->contact_world, B->n_contacts, w, &R.c0, &R.c1);
    return R;
}

static int world_rows(const orc_batch *B, const world_range *R) {
    int m = 0;
    for (int j = R->j0; j < R->j1; ++j) m += joint_rows(B->joint_type[j]);
    for (int j = R->j0; j < R->j1; ++j) m += has_limit(B->joint_limit + 2 * (size_t)j);
    for (int j = R->j0; j < R->j1; ++j) m += has_drive(B, j);
    m += 3 * (R->c1 - R->c0);
    return m;
}

static void sys_free(world_sys *S) {
    free(S->J);
    free(S->f);
    free(S->vstar);
    free(S->kind);
    free(S->mu);
    free(S->Minv);
    free(S->uf);
    free(S->Rreg);
}

/* Body quantities (Sec. 3, Eq. 1 and the Newton-Euler forces h) and the
 * rows of one world at the configuration q; v* per Sec. 3 Baumgarte
 * stabilisation.  hz is the time from q to the end of the step over which
 * the position-level terms act: dt for semi-implicit Euler, dt / 2 for the
 * Moreau-Jean midpoint (q is then the half-step configuration). */
static int build_world(const orc_batch *B, const orc_params *P, const double *q, const double *u,
                       const double *joint_torque, int w, double hz, world_sys *S) {
    world_range R = get_range(B, w);
    S->b0 = R.b0;
    S->nb = R.b1 - R.b0;
    S->m = world_rows(B, &R);
    int nb = S->nb, m = S->m, n6 = 6 * nb;
    S->J = calloc((size_t)m * n6 + 1, sizeof(double));
    S->f = calloc((size_t)m + 1, sizeof(double));
    S->vstar = calloc((size_t)m + 1, sizeof(double));
    S->kind = calloc((size_t)m + 1, sizeof(int));
    S->mu = calloc((size_t)m + 1, sizeof(double));
    S->Minv = calloc((size_t)nb * 36 + 1, sizeof(double));
    S->uf = calloc((size_t)n6 + 1, sizeof(double));
    S->Rreg = calloc((size_t)m + 1, sizeof(double));
    if (!S->J || !S->f || !S->vstar || !S->kind || !S->mu || !S->Minv || !S->uf || !S->Rreg) return -1;

    /* generalized forces h: gravity, gyroscopic, joint actuation */
    double *hw = calloc((size_t)n6 + 1, sizeof(double));
    double *Iw = calloc((size_t)nb * 9 + 1, sizeof(double));
    for (int i = 0; i < nb; ++i) {
        int gb = R.b0 + i;
        const double *qi = q + 7 * (size_t)gb, *ui = u + 6 * (size_t)gb;
        double Rm[9];
        quat_to_rot(qi + 3, Rm);
        const double *Ib = B->inertia + 3 * (size_t)gb;
        double m_i = B->mass[gb];
        /* I_w = R I_b R^T and its inverse R I_b^-1 R^T (Eq. 1) */
        double *Mi = S->Minv + 36 * (size_t)i;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0, si = 0.0;
                for (int k = 0; k < 3; ++k) {
                    s += Rm[3 * r + k] * Ib[k] * Rm[3 * c + k];
                    si += Rm[3 * r + k] / Ib[k] * Rm[3 * c + k];
                }
                Iw[9 * i + 3 * r + c] = s;
                Mi[6 * (3 + r) + 3 + c] = si;
            }
        for (int k = 0; k < 3; ++k) Mi[6 * k + k] = 1.0 / m_i;
        /* h = (m g, -w x I_w w) */
        double Iww[3], gyro[3];
        mat_vec3(Iw + 9 * i, ui + 3, Iww);
        cross3(ui + 3, Iww, gyro);
        for (int k = 0; k < 3; ++k) {
            hw[6 * i + k] = m_i * P->gravity[k];
            hw[6 * i + 3 + k] = -gyro[k];
        }
    }
    if (joint_torque) {
        for (int j = R.j0; j < R.j1; ++j) {
            double tau = joint_torque[j];
            if (tau == 0.0) continue;
            double Ja[6], Jb[6];
            joint_coordinate(B, q, j, Ja, Jb);
            int la = local_body(B->joint_body[2 * j], S->b0);
            int lb = local_body(B->joint_body[2 * j + 1], S->b0);
            for (int k = 0; k < 6; ++k) {
                if (la >= 0) hw[6 * la + k] += tau * Ja[k];
                if (lb >= 0) hw[6 * lb + k] += tau * Jb[k];
            }
        }
    }
    /* free velocity of the bodies: u_f = u + dt M^-1 h */
    for (int i = 0; i < nb; ++i) {
        const double *ui = u + 6 * (size_t)(R.b0 + i);
        const double *Mi = S->Minv + 36 * (size_t)i;
        for (int r = 0; r < 6; ++r) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += Mi[6 * r + c] * hw[6 * i + c];
            S->uf[6 * i + r] = ui[r] + P->dt * s;
        }
    }
    free(hw);
    free(Iw);

    /* rows: joints, then limits, then drives, then contacts */
    int r = 0;
    for (int j = R.j0; j < R.j1; ++j) {
        assemble_joint(B, q, j, S, r);
        r += joint_rows(B->joint_type[j]);
    }
    for (int j = R.j0; j < R.j1; ++j)
        if (has_limit(B->joint_limit + 2 * (size_t)j)) assemble_limit(B, q, j, S, r++);
    const int r_drive0 = r;
    for (int j = R.j0; j < R.j1; ++j)
        if (has_drive(B, j)) {
            double Ja[6], Jb[6];
            joint_coordinate(B, q, j, Ja, Jb);
            put_row(S, r, local_body(B->joint_body[2 * j], S->b0), Ja, local_body(B->joint_body[2 * j + 1], S->b0),
                    Jb);
            S->kind[r] = ORC_ROW_BILATERAL;
            ++r;
        }
    const int r_drive1 = r;
    for (int c = R.c0; c < R.c1; ++c) {
        assemble_contact(B, q, c, S, r);
        r += 3;
    }
    /* Baumgarte bias: bilateral rows beta f / hz; unilateral rows f / hz
     * while separated (speculative) and beta f / hz when penetrating. */
    for (int i = 0; i < m; ++i) {
        double fi = S->f[i];
        switch (S->kind[i]) {
        case ORC_ROW_BILATERAL: S->vstar[i] = P->baumgarte * fi / hz; break;
        case ORC_ROW_LIMIT:
        case ORC_ROW_NORMAL: S->vstar[i] = (fi >= 0.0 ? fi : P->baumgarte * fi) / hz; break;
        default: S->vstar[i] = 0.0;
        }
    }
    /* Joint-space drive rows (Sec. 3 implicit PD, armature, viscous
     * damping; Eq. 2 R and v*).  Along the joint coordinate c with rate
     * cdot = J_c u the drive applies, over the step, the impulse
     *   lambda = dt [kp (ref - c - hz cdot+) - (kd + d) cdot+
     *                - I_a (cdot+ - cdot-) / dt],
     * PD on the coordinate reached at the end of the step (c + hz cdot+),
     * damping on the new rate, the rotor inertia I_a opposing the change of
     * rate.  Solved for cdot+ with K = kp hz + kd + d + I_a / dt:
     *   J_c u+ + lambda / (dt K) - (kp (ref - c) + I_a cdot- / dt) / K = 0,
     * a bilateral row with R = 1 / (dt K) and v* = -(kp (ref - c) +
     * I_a cdot- / dt) / K. */
    {
        int rr = r_drive0;
        for (int j = R.j0; j < R.j1 && rr < r_drive1; ++j) {
            if (!has_drive(B, j)) continue;
            const double *d = B->joint_drive + 5 * (size_t)j;
            const double kp = d[0], kd = d[1], damp = d[2], arm = d[3], ref = d[4];
            double Ja[6], Jb[6];
            const double c = joint_coordinate(B, q, j, Ja, Jb);
            const int a = B->joint_body[2 * j], b = B->joint_body[2 * j + 1];
            double rate = 0.0;
            for (int k = 0; k < 6; ++k) {
                rate += Ja[k] * u[6 * (size_t)a + k];
                if (b >= 0) rate += Jb[k] * u[6 * (size_t)b + k];
            }
            const double K = kp * hz + kd + damp + arm / P->dt;
            S->Rreg[rr] = 1.0 / (P->dt * K);
            S->vstar[rr] = -(kp * (ref - c) + arm * rate / P->dt) / K;
            S->f[rr] = 0.0;
            ++rr;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. 4: Delassus matrix and free velocity                                 */
/* ------------------------------------------------------------------------ */

static void delassus(const world_sys *S, double *D, double *vf) {
    int m = S->m, n6 = 6 * S->nb;
    double *MJt = calloc((size_t)n6 * m + 1, sizeof(double)); /* [n6][m] */
    for (int i = 0; i < S->nb; ++i)
        for (int r = 0; r < 6; ++r)
            for (int k = 0; k < m; ++k) {
                double s = 0.0;
                for (int c = 0; c < 6; ++c) s += S->Minv[36 * i + 6 * r + c] * S->J[(size_t)k * n6 + 6 * i + c];
                MJt[(size_t)(6 * i + r) * m + k] = s;
            }
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            double s = 0.0;
            for (int c = 0; c < n6; ++c) s += S->J[(size_t)a * n6 + c] * MJt[(size_t)c * m + b];
            D[(size_t)a * m + b] = s;
        }
    for (int a = 0; a < m; ++a) D[(size_t)a * m + a] += S->Rreg[a]; /* D = J M^-1 J^T + R */
    for (int a = 0; a < m; ++a) {
        double s = 0.0;
        for (int c = 0; c < n6; ++c) s += S->J[(size_t)a * n6 + c] * S->uf[c];
        vf[a] = s + S->vstar[a];
    }
    free(MJt);
}

/* ------------------------------------------------------------------------ */
/* cones (Sec. 3): free rows, R+ for limits, Coulomb cone for contacts       */
/* ------------------------------------------------------------------------ */

/* Euclidean projection onto K_mu = {(l_n, l_t): |l_t| <= mu l_n} (the
 * textbook second-order-cone projection). */
static void project_coulomb(double mu, const double *w, double *o) {
    double tn = sqrt(w[1] * w[1] + w[2] * w[2]);
    double wn = w[0];
    if (tn <= mu * wn) {
        o[0] = w[0];
        o[1] = w[1];
        o[2] = w[2];
    } else if (mu * tn <= -wn) {
        o[0] = o[1] = o[2] = 0.0;
    } else {
        double ln = (mu * tn + wn) / (1.0 + mu * mu);
        double s = tn > 0.0 ? mu * ln / tn : 0.0;
        o[0] = ln;
        o[1] = s * w[1];
        o[2] = s * w[2];
    }
}

/* Projection onto K (row kinds give the block structure). */
static void project_K(int m, const int *kind, const double *mu, const double *w, double *o) {
    for (int i = 0; i < m;) {
        if (kind[i] == ORC_ROW_NORMAL) {
            project_coulomb(mu[i], w + i, o + i);
            i += 3;
        } else if (kind[i] == ORC_ROW_LIMIT) {
            o[i] = w[i] > 0.0 ? w[i] : 0.0;
            i += 1;
        } else {
            o[i] = w[i];
            i += 1;
        }
    }
}

/* De Saxce correction Gamma(w): (mu |w_t|, 0, 0) per contact, 0 elsewhere
 * (Sec. 4, Eq. 3). */
static void desaxce(int m, const int *kind, const double *mu, const double *w, double *o) {
    for (int i = 0; i < m; ++i) o[i] = 0.0;
    for (int i = 0; i < m; ++i)
        if (kind[i] == ORC_ROW_NORMAL) o[i] = mu[i] * sqrt(w[i + 1] * w[i + 1] + w[i + 2] * w[i + 2]);
}

/* ------------------------------------------------------------------------ */
/* Cholesky (textbook, column by column) and triangular solves               */
/* ------------------------------------------------------------------------ */

int orc_cholesky(int n, const double *A, double *L) {
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) return -1 - j;
        double d = sqrt(s);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / d;
        }
    }
    return 0;
}

/* solve L L^T x = b */
static void chol_solve(int n, const double *L, const double *b, double *x) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/* Sec. 5.1 iterative solve of A x = b for the SPD A = D~ + diag(eta + rho):
 * Conjugate Residual (Saad, Iterative Methods for Sparse Linear Systems,
 * Alg. 6.20) from the initial guess in x, exactly n_it iterations (fewer if
 * the residual vanishes).  A is applied as a plain product. */
static void cr_solve(int n, const double *A, const double *b, int n_it, double *x, double *work) {
    double *r = work, *p = work + n, *Ar = work + 2 * (size_t)n, *Ap = work + 3 * (size_t)n;
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = 0; j < n; ++j) s -= A[(size_t)i * n + j] * x[j];
        r[i] = s;
        p[i] = s;
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * r[j];
        Ar[i] = s;
        Ap[i] = s;
    }
    double rAr = 0.0;
    for (int i = 0; i < n; ++i) rAr += r[i] * Ar[i];
    for (int k = 0; k < n_it; ++k) {
        double ApAp = 0.0;
        for (int i = 0; i < n; ++i) ApAp += Ap[i] * Ap[i];
        if (!(ApAp > 0.0) || !(rAr > 0.0)) break;
        const double alpha = rAr / ApAp;
        for (int i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += A[(size_t)i * n + j] * r[j];
            Ar[i] = s;
        }
        double rAr_new = 0.0;
        for (int i = 0; i < n; ++i) rAr_new += r[i] * Ar[i];
        const double beta = rAr_new / rAr;
        rAr = rAr_new;
        for (int i = 0; i < n; ++i) {
            p[i] = r[i] + beta * p[i];
            Ap[i] = Ar[i] + beta * Ap[i];
        }
    }
}

static double inf_norm(int n, const double *v) {
    double r = 0.0;
    for (int i = 0; i < n; ++i) {
        double a = fabs(v[i]);
        if (a > r || isnan(a)) r = a;
    }
    return r;
}

/* ------------------------------------------------------------------------ */
/* Sec. 4.1 Jacobi preconditioner: p_i = D_ii^-1/2 on bilateral and limit   */
/* rows; one scalar per contact, (trace of the 3x3 block / 3)^-1/2, so that */
/* the Coulomb cone, Gamma and the NCP keep their form after scaling.        */
/* ------------------------------------------------------------------------ */

static void preconditioner(int m, const double *D, const int *kind, int enabled, double *p) {
    for (int i = 0; i < m; ++i) p[i] = 1.0;
    if (!enabled) return;
    for (int i = 0; i < m;) {
        if (kind[i] == ORC_ROW_NORMAL) {
            double t = (D[(size_t)i * m + i] + D[(size_t)(i + 1) * m + i + 1] + D[(size_t)(i + 2) * m + i + 2]) / 3.0;
            double s = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
            p[i] = p[i + 1] = p[i + 2] = s;
            i += 3;
        } else {
            double t = D[(size_t)i * m + i];
            p[i] = t > 0.0 ? 1.0 / sqrt(t) : 1.0;
            i += 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: Proximal-ADMM on the (preconditioned) dual problem                */
/* ------------------------------------------------------------------------ */

/* Solve one dual NCP given D (m x m, physical), v_f, row kinds and mu.
 * lambda_ws: physical warm start or NULL.  Returns the status; writes
 * lambda (physical), lambda_tilde (scaled y, may be NULL), iteration count
 * and the residuals (r_p, r_d, r_c in scaled units; r_ncp at the returned
 * iterate). */
int orc_solve_ncp(int m, const double *D, const double *vf, const int *kind, const double *mu,
                  const orc_params *P, const double *lambda_ws, double *lambda, double *lambda_tilde,
                  int *iters_out, double *resid, const uint8_t *replay_log, uint8_t *log_out) {
    int status = ORC_OK;
    if (m == 0) {
        *iters_out = 0;
        for (int k = 0; k < 4; ++k) resid[k] = 0.0;
        return status;
    }
    size_t mm = (size_t)m * m;
    double *p = malloc(sizeof(double) * m);
    double *Dt = malloc(sizeof(double) * mm);
    double *A = malloc(sizeof(double) * mm);
    double *L = malloc(sizeof(double) * mm);
    double *vt = malloc(sizeof(double) * m);
    double *rho = malloc(sizeof(double) * m);
    double *x = calloc(m, sizeof(double)), *y = calloc(m, sizeof(double)), *z = calloc(m, sizeof(double));
    double *yh = calloc(m, sizeof(double)), *zh = calloc(m, sizeof(double));
    double *yp = calloc(m, sizeof(double)), *zp = calloc(m, sizeof(double));
    double *s = calloc(m, sizeof(double)), *rhs = calloc(m, sizeof(double));
    double *xn = calloc(m, sizeof(double)), *yn = calloc(m, sizeof(double)), *zn = calloc(m, sizeof(double));
    double *v = calloc(m, sizeof(double)), *g = calloc(m, sizeof(double)), *tmp = calloc(m, sizeof(double));

    /* scaled system: D~ = P D P, v~_f = P v_f */
    preconditioner(m, D, kind, P->precond, p);
    for (int i = 0; i < m; ++i) {
        vt[i] = p[i] * vf[i];
        rho[i] = kind[i] == ORC_ROW_BILATERAL ? P->rho_bil : P->rho_c;
        for (int j = 0; j < m; ++j) Dt[(size_t)i * m + j] = p[i] * D[(size_t)i * m + j] * p[j];
    }
    /* Alg. 1, step 1: D_{eta,rho} = D~ + diag(eta + rho), factored once */
    for (size_t k = 0; k < mm; ++k) A[k] = Dt[k];
    for (int i = 0; i < m; ++i) A[(size_t)i * m + i] += P->eta + rho[i];
    double *crw = P->cr_iters > 0 ? malloc(sizeof(double) * 4 * (size_t)m) : NULL;
    if (P->cr_iters <= 0 && orc_cholesky(m, A, L) != 0) {
        status |= ORC_FACTOR_FAIL;
        for (int i = 0; i < m; ++i) {
            lambda[i] = 0.0;
            if (lambda_tilde) lambda_tilde[i] = 0.0;
        }
        *iters_out = 0;
        resid[0] = resid[1] = resid[2] = resid[3] = NAN;
        goto done;
    }

    /* Alg. 1, step 2: initial iterate.  Cold: zeros.  Warm: y = x =
     * Pi_K(P^-1 lambda_ws) and z = v~(y) + Gamma(v~(y)) on unilateral rows,
     * z = 0 on bilateral rows (the dual cone of a free row is {0}). */
    if (P->warmstart && lambda_ws) {
        for (int i = 0; i < m; ++i) tmp[i] = lambda_ws[i] / p[i];
        project_K(m, kind, mu, tmp, y);
        for (int i = 0; i < m; ++i) {
            double a = vt[i];
            for (int j = 0; j < m; ++j) a += Dt[(size_t)i * m + j] * y[j];
            v[i] = a;
        }
        desaxce(m, kind, mu, v, g);
        for (int i = 0; i < m; ++i) {
            x[i] = y[i];
            z[i] = kind[i] == ORC_ROW_BILATERAL ? 0.0 : v[i] + g[i];
        }
    }
    for (int i = 0; i < m; ++i) {
        yh[i] = yp[i] = y[i];
        zh[i] = zp[i] = z[i];
    }

    double a_k = 1.0;
    double c_prev = INFINITY;
    int N = P->fixed_iters > 0 ? P->fixed_iters : P->max_iters;
    int n_uni = 0; /* limit and contact rows: the rows an adaptive penalty acts on */
    for (int i = 0; i < m; ++i) n_uni += kind[i] != ORC_ROW_BILATERAL;
    int it = 0;
    double rp = INFINITY, rd = INFINITY, rc = INFINITY;
    int converged = 0;
    for (it = 1; it <= N; ++it) {
        /* step 4: De Saxce correction at the previous (extrapolated) dual */
        desaxce(m, kind, mu, zh, s);
        /* step 5: x = D_{eta,rho}^-1 (-v_f - s + eta x + rho y + z) */
        for (int i = 0; i < m; ++i) rhs[i] = -vt[i] - s[i] + P->eta * x[i] + rho[i] * yh[i] + zh[i];
        if (P->cr_iters > 0) {
            /* warm start at the previous iterate (Sec. 5.1) */
            for (int i = 0; i < m; ++i) xn[i] = x[i];
            cr_solve(m, A, rhs, P->cr_iters, xn, crw);
        } else {
            chol_solve(m, L, rhs, xn);
        }
        /* step 6: y = Pi_K(x - z / rho) */
        for (int i = 0; i < m; ++i) tmp[i] = xn[i] - zh[i] / rho[i];
        project_K(m, kind, mu, tmp, yn);
        /* step 7: z = z - rho (x - y) */
        for (int i = 0; i < m; ++i) zn[i] = zh[i] - rho[i] * (xn[i] - yn[i]);

        /* step 9 residuals at (x, y, z): primal x - y; dual: the corrected
         * constraint velocity v~ + Gamma(v~) against z; complementarity
         * y . (v~ + Gamma(v~)) per unilateral block. */
        for (int i = 0; i < m; ++i) {
            double a = vt[i];
            for (int j = 0; j < m; ++j) a += Dt[(size_t)i * m + j] * xn[j];
            v[i] = a;
        }
        desaxce(m, kind, mu, v, g);
        rp = 0.0;
        rd = 0.0;
        rc = 0.0;
        for (int i = 0; i < m; ++i) {
            double e1 = fabs(xn[i] - yn[i]);
            double e2 = fabs(v[i] + g[i] - zn[i]);
            if (!(e1 <= rp)) rp = e1;
            if (!(e2 <= rd)) rd = e2;
        }
        for (int i = 0; i < m;) {
            if (kind[i] == ORC_ROW_NORMAL) {
                double c = fabs(yn[i] * (v[i] + g[i]) + yn[i + 1] * v[i + 1] + yn[i + 2] * v[i + 2]);
                if (!(c <= rc)) rc = c;
                i += 3;
            } else if (kind[i] == ORC_ROW_LIMIT) {
                double c = fabs(yn[i] * v[i]);
                if (!(c <= rc)) rc = c;
                i += 1;
            } else {
                i += 1;
            }
        }

        /* step 8: Nesterov extrapolation of (y, z) with adaptive restart
         * (fast ADMM with restart, Goldstein, O'Donoghue, Setzer and
         * Baraniuk, SIAM J. Imaging Sci. 2014): combined residual
         * c = |y - y^|^2_rho + |z - z^|^2_{1/rho}. */
        if (P->accel) {
            double c = 0.0;
            for (int i = 0; i < m; ++i) {
                double dy = yn[i] - yh[i], dz = zn[i] - zh[i];
                c += rho[i] * dy * dy + dz * dz / rho[i];
            }
            int restart;
            if (P->replay && replay_log) restart = (replay_log[it - 1] & 1) != 0;
            else restart = !(c < P->restart_factor * c_prev);
            /* the log holds log_stride decisions per world (0: as many as iterations) */
            if (log_out && (P->log_stride <= 0 || it <= P->log_stride)) log_out[it - 1] = (uint8_t)restart;
            if (!restart) {
                double a_next = 0.5 * (1.0 + sqrt(1.0 + 4.0 * a_k * a_k));
                double beta = (a_k - 1.0) / a_next;
                for (int i = 0; i < m; ++i) {
                    yh[i] = yn[i] + beta * (yn[i] - yp[i]);
                    zh[i] = zn[i] + beta * (zn[i] - zp[i]);
                }
                a_k = a_next;
                c_prev = c;
            } else {
                for (int i = 0; i < m; ++i) {
                    yh[i] = yp[i];
                    zh[i] = zp[i];
                }
                a_k = 1.0;
                c_prev = c_prev / P->restart_factor;
            }
        } else {
            for (int i = 0; i < m; ++i) {
                yh[i] = yn[i];
                zh[i] = zn[i];
            }
        }
        for (int i = 0; i < m; ++i) {
            x[i] = xn[i];
            y[i] = yn[i];
            z[i] = zn[i];
            yp[i] = yn[i];
            zp[i] = zn[i];
        }
        if (!(isfinite(rp) && isfinite(rd) && isfinite(rc))) {
            status |= ORC_NONFINITE;
            break;
        }
        /* step 10: exit when all three residuals are below eps */
        if (P->fixed_iters <= 0 && rp < P->eps && rd < P->eps && rc < P->eps) {
            converged = 1;
            break;
        }
        /* Adaptive penalty on the limit and contact rows (not in the paper,
         * whose penalty is fixed: residual balancing after Boyd, Parikh, Chu,
         * Peleato and Eckstein 2011, Sec. 3.4.1, here on the unilateral rows'
         * share of a per-row penalty).  At the checkpoint iterations
         * first, 2 first, 4 first, ...: when r_d > tau r_p the unilateral
         * penalty is divided by f, when r_p > tau r_d it is multiplied by f.
         * A change refactors D~ + diag(eta + rho) and restarts the
         * acceleration from the current iterate (a = 1, y^ = y, z^ = z);
         * x, y and z carry over (z is not scaled by rho).  The decision is
         * logged in bits 1 (lowered) and 2 (raised) of the iteration's log
         * byte and read from there in replay. */
        if (P->adapt_ratio > 0.0 && n_uni > 0 && P->adapt_first > 0 && it >= P->adapt_first &&
            it % P->adapt_first == 0 && ((it / P->adapt_first) & (it / P->adapt_first - 1)) == 0) {
            int dir = 0;
            if (P->replay && replay_log) dir = (replay_log[it - 1] >> 1) & 3;
            else if (rd > P->adapt_ratio * rp) dir = 1;
            else if (rp > P->adapt_ratio * rd) dir = 2;
            if (log_out && (P->log_stride <= 0 || it <= P->log_stride)) log_out[it - 1] |= (uint8_t)(dir << 1);
            if (dir == 1 || dir == 2) {
                const double f = dir == 1 ? 1.0 / P->adapt_factor : P->adapt_factor;
                for (int i = 0; i < m; ++i)
                    if (kind[i] != ORC_ROW_BILATERAL) rho[i] *= f;
                for (size_t k = 0; k < mm; ++k) A[k] = Dt[k];
                for (int i = 0; i < m; ++i) A[(size_t)i * m + i] += P->eta + rho[i];
                if (P->cr_iters <= 0 && orc_cholesky(m, A, L) != 0) {
                    status |= ORC_FACTOR_FAIL;
                    break;
                }
                a_k = 1.0;
                c_prev = INFINITY;
                for (int i = 0; i < m; ++i) {
                    yh[i] = y[i];
                    zh[i] = z[i];
                }
            }
        }
    }
    if (it > N) it = N;
    if (P->fixed_iters <= 0 && !converged && !(status & ORC_NONFINITE)) status |= ORC_MAXITER;
    *iters_out = it;

    /* step 11: lambda = P y; NCP natural-map residual at y */
    for (int i = 0; i < m; ++i) {
        double a = vt[i];
        for (int j = 0; j < m; ++j) a += Dt[(size_t)i * m + j] * y[j];
        v[i] = a;
    }
    desaxce(m, kind, mu, v, g);
    for (int i = 0; i < m; ++i) tmp[i] = y[i] - (v[i] + g[i]);
    project_K(m, kind, mu, tmp, s);
    for (int i = 0; i < m; ++i) s[i] = y[i] - s[i];
    resid[0] = rp;
    resid[1] = rd;
    resid[2] = rc;
    resid[3] = inf_norm(m, s);
    for (int i = 0; i < m; ++i) {
        lambda[i] = p[i] * y[i];
        if (lambda_tilde) lambda_tilde[i] = y[i];
    }

done:
    free(crw);
    free(p); free(Dt); free(A); free(L); free(vt); free(rho);
    free(x); free(y); free(z); free(yh); free(zh); free(yp); free(zp);
    free(s); free(rhs); free(xn); free(yn); free(zn); free(v); free(g); free(tmp);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3 semi-implicit Euler: u+ = u_f + M^-1 J^T lambda; poses explicit   */
/* with u+, orientation by the exponential map (left multiplication, world  */
/* angular velocity), then renormalised.                                     */
/* ------------------------------------------------------------------------ */

/* Pose update over the time hz with u+ from the configuration q (the
 * pre-step pose for semi-implicit Euler, hz = dt; the half-step pose for
 * the Moreau-Jean midpoint, hz = dt / 2). */
static void advance_pose(const double *qi, const double *un, double hz, double *qo) {
    for (int k = 0; k < 3; ++k) qo[k] = qi[k] + hz * un[k];
    double wn = sqrt(un[3] * un[3] + un[4] * un[4] + un[5] * un[5]);
    double dq[4] = {0, 0, 0, 1};
    if (wn > 0.0) {
        double half = 0.5 * hz * wn;
        double sh = sin(half) / wn;
        dq[0] = un[3] * sh;
        dq[1] = un[4] * sh;
        dq[2] = un[5] * sh;
        dq[3] = cos(half);
    }
    double qn[4];
    quat_mul(dq, qi + 3, qn);
    double nn = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
    for (int k = 0; k < 4; ++k) qo[3 + k] = qn[k] / nn;
}

static void integrate(const world_sys *S, const orc_params *P, const double *q, const double *lam, double hz,
                      double *q_out, double *u_out) {
    int nb = S->nb, m = S->m, n6 = 6 * nb;
    for (int i = 0; i < nb; ++i) {
        double imp[6] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < 6; ++k)
            for (int r = 0; r < m; ++r) imp[k] += S->J[(size_t)r * n6 + 6 * i + k] * lam[r];
        double un[6];
        for (int r = 0; r < 6; ++r) {
            double s = 0.0;
            for (int c = 0; c < 6; ++c) s += S->Minv[36 * (size_t)i + 6 * r + c] * imp[c];
            un[r] = S->uf[6 * i + r] + s;
        }
        int gb = S->b0 + i;
        for (int k = 0; k < 6; ++k) u_out[6 * (size_t)gb + k] = un[k];
        advance_pose(q + 7 * (size_t)gb, un, hz, q_out + 7 * (size_t)gb);
    }
    (void)P;
}

/* The configuration the step's constraints and forces are evaluated at:
 * the pre-step poses (semi-implicit Euler), or (Moreau-Jean midpoint) the
 * poses advanced by dt / 2 with the pre-step twists, written to qm for the
 * bodies of world w.  Returns the horizon hz from there to the step's end. */
static double step_configuration(const orc_batch *B, const orc_params *P, const double *q, const double *u, int w,
                                 double *qm) {
    world_range R = get_range(B, w);
    const int mj = P->integrator == 1;
    for (int gb = R.b0; gb < R.b1; ++gb) {
        if (mj) advance_pose(q + 7 * (size_t)gb, u + 6 * (size_t)gb, 0.5 * P->dt, qm + 7 * (size_t)gb);
        else
            for (int k = 0; k < 7; ++k) qm[7 * (size_t)gb + k] = q[7 * (size_t)gb + k];
    }
    return mj ? 0.5 * P->dt : P->dt;
}

/* ------------------------------------------------------------------------ */
/* public entry points                                                       */
/* ------------------------------------------------------------------------ */

/* Row count of every world (row_offset[nw+1]). */
void orc_row_offsets(const orc_batch *B, int64_t *row_offset) {
    row_offset[0] = 0;
    for (int w = 0; w < B->n_worlds; ++w) {
        world_range R = get_range(B, w);
        row_offset[w + 1] = row_offset[w] + world_rows(B, &R);
    }
}

/* One full time step of every world (worlds in parallel when built with
 * OpenMP).  Returns 0, or -1 on allocation failure. */
int orc_step(const orc_batch *B, const orc_params *P, orc_io *io) {
    int nw = B->n_worlds;
    orc_row_offsets(B, io->row_offset);
    int err = 0;
    /* configuration of the constraints (pre-step or half-step poses) */
    double *qm = malloc(sizeof(double) * (7 * (size_t)B->n_bodies + 1));
    if (!qm) return -1;
#pragma omp parallel for schedule(static)
    for (int w = 0; w < nw; ++w) {
        world_sys S;
        memset(&S, 0, sizeof S);
        const double hz = step_configuration(B, P, io->q, io->u, w, qm);
        if (build_world(B, P, qm, io->u, io->joint_torque, w, hz, &S) != 0) {
            err = -1;
            sys_free(&S);
            continue;
        }
        int m = S.m;
        int64_t r0 = io->row_offset[w];
        double *D = malloc(sizeof(double) * ((size_t)m * m + 1));
        double *vf = malloc(sizeof(double) * ((size_t)m + 1));
        delassus(&S, D, vf);
        int it = 0;
        const uint8_t *rlog = io->restart_log && P->replay ? io->restart_log + (size_t)w * P->log_stride : NULL;
        uint8_t *wlog = io->restart_log && !P->replay ? io->restart_log + (size_t)w * P->log_stride : NULL;
        int st = orc_solve_ncp(m, D, vf, S.kind, S.mu, P, io->lambda_ws ? io->lambda_ws + r0 : NULL,
                               io->lambda + r0, io->lambda_tilde ? io->lambda_tilde + r0 : NULL, &it,
                               io->resid + 4 * (size_t)w, rlog, wlog);
        io->iters[w] = it;
        io->status[w] = st;
        integrate(&S, P, qm, io->lambda + r0, hz, io->q_out, io->u_out);
        free(D);
        free(vf);
        sys_free(&S);
    }
    free(qm);
    return err;
}

/* Conjugate Residual on an explicit SPD system (for tests): n_it
 * iterations from the initial guess in x. */
int orc_cr_solve(int n, const double *A, const double *b, int n_it, double *x) {
    double *w = malloc(sizeof(double) * 4 * (size_t)(n > 0 ? n : 1));
    if (!w) return -1;
    cr_solve(n, A, b, n_it, x, w);
    free(w);
    return 0;
}

/* Threads of the OpenMP loops over worlds (for timing the oracle on one
 * core and on all of them). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Dimensions of world w: bodies and rows. */
void orc_world_dims(const orc_batch *B, int w, int *nb, int *m) {
    world_range R = get_range(B, w);
    *nb = R.b1 - R.b0;
    *m = world_rows(B, &R);
}

/* The assembled system of world w, for tests: J [m x 6nb], f, v*, kinds,
 * mu, the 6x6 blocks of M^-1 [nb x 36], u_f [6nb], D [m x m], v_f [m]. */
int orc_world_system(const orc_batch *B, const orc_params *P, const double *q, const double *u,
                     const double *joint_torque, int w, double *J, double *f, double *vstar, int *kind,
                     double *mu, double *Minv, double *uf, double *D, double *vf, double *Rreg) {
    world_sys S;
    memset(&S, 0, sizeof S);
    double *qm = malloc(sizeof(double) * (7 * (size_t)B->n_bodies + 1));
    if (!qm) return -1;
    const double hz = step_configuration(B, P, q, u, w, qm);
    int bad = build_world(B, P, qm, u, joint_torque, w, hz, &S) != 0;
    free(qm);
    if (bad) {
        sys_free(&S);
        return -1;
    }
    int m = S.m, n6 = 6 * S.nb;
    memcpy(J, S.J, sizeof(double) * (size_t)m * n6);
    memcpy(f, S.f, sizeof(double) * m);
    memcpy(vstar, S.vstar, sizeof(double) * m);
    memcpy(kind, S.kind, sizeof(int) * m);
    memcpy(mu, S.mu, sizeof(double) * m);
    memcpy(Minv, S.Minv, sizeof(double) * 36 * S.nb);
    memcpy(uf, S.uf, sizeof(double) * n6);
    if (Rreg) memcpy(Rreg, S.Rreg, sizeof(double) * m);
    delassus(&S, D, vf);
    sys_free(&S);
    return 0;
}

/* The poses the step's constraints are evaluated at (q itself, or the
 * Moreau-Jean half-step poses) for every world, into qm [nb*7]. */
void orc_step_configuration(const orc_batch *B, const orc_params *P, const double *q, const double *u, double *qm) {
    for (int w = 0; w < B->n_worlds; ++w) (void)step_configuration(B, P, q, u, w, qm);
}

/* Joint coordinate of joint j and its two 6-vector Jacobians. */
double orc_joint_coordinate(const orc_batch *B, const double *q, int j, double *Ja, double *Jb) {
    return joint_coordinate(B, q, j, Ja, Jb);
}

/* Cone projection of one block: kind 0 free (1 value), 1 R+ (1 value),
 * 2 Coulomb cone (3 values). */
void orc_project_block(int kind, double mu, const double *w, double *o) {
    if (kind == ORC_ROW_NORMAL) project_coulomb(mu, w, o);
    else if (kind == ORC_ROW_LIMIT) o[0] = w[0] > 0.0 ? w[0] : 0.0;
    else o[0] = w[0];
}

/* Triangular-basis of a normal, for tests. */
void orc_tangent_basis(const double *n, double *t1, double *t2) { tangent_basis(n, t1, t2); }

/* ------------------------------------------------------------------------ */
/* Sec. 6.3 forward kinematics: poses consistent with every joint constraint */
/* and with target joint coordinates, by Gauss-Newton                        */
/* ------------------------------------------------------------------------ */

/* For every world w: starting from q_in, find poses with f(q) = 0 for every
 * joint (Sec. 3 constraint functions) and c_j(q) = target[j] for every
 * joint with a finite target (NaN = free), keeping body base[w] fixed (-1:
 * none).  Gauss-Newton on F = (f, c_T - target) with J its Jacobian over
 * the body twists: each iteration takes the least-change step
 *   Delta = -W J^T (J W J^T + mu I)^-1 F,   W = M^-1 (base block 0),
 * mu = 1e-12 times the largest diagonal entry of J W J^T (the loop rows of
 * planar loops are redundant), and moves every body by Delta with the
 * exponential map (r += Delta_v, R <- exp(Delta_w) R).  It stops when
 * |F|_inf <= tol (iters = iterations taken) or after max_iters.  resid[w]
 * = |F|_inf at the returned poses.  Limits, drives and contacts play no
 * part.  Returns 0, or -1 on allocation failure. */
int orc_fk(const orc_batch *B, const double *q_in, const double *target, const int32_t *base, double tol,
           int max_iters, double *q_out, int32_t *iters, double *resid) {
    orc_batch Bj = *B; /* joints only: no contacts, no drive rows */
    Bj.n_contacts = 0;
    Bj.joint_drive = NULL;
    orc_params P;
    memset(&P, 0, sizeof P);
    P.dt = 1.0;
    memcpy(q_out, q_in, sizeof(double) * 7 * (size_t)B->n_bodies);
    int err = 0;
#pragma omp parallel for schedule(dynamic)
    for (int w = 0; w < B->n_worlds; ++w) {
        world_range R = get_range(&Bj, w);
        const int nb = R.b1 - R.b0, n6 = 6 * nb;
        int nt = 0;
        for (int j = R.j0; j < R.j1; ++j) nt += !isnan(target[j]);
        const int mj = 5 * (R.j1 - R.j0), m = mj + nt;
        double *u0 = calloc((size_t)6 * B->n_bodies + 1, sizeof(double));
        double *Jt = calloc((size_t)m * n6 + 1, sizeof(double)), *F = calloc((size_t)m + 1, sizeof(double));
        double *WJ = calloc((size_t)n6 * m + 1, sizeof(double)), *A = calloc((size_t)m * m + 1, sizeof(double));
        double *L = calloc((size_t)m * m + 1, sizeof(double)), *y = calloc((size_t)m + 1, sizeof(double));
        double *Dl = calloc((size_t)n6 + 1, sizeof(double));
        if (!u0 || !Jt || !F || !WJ || !A || !L || !y || !Dl) {
            err = -1;
        } else {
            int it = 0;
            double fn = INFINITY;
            for (;;) {
                world_sys S;
                memset(&S, 0, sizeof S);
                if (build_world(&Bj, &P, q_out, u0, NULL, w, 1.0, &S) != 0) {
                    err = -1;
                    sys_free(&S);
                    break;
                }
                /* F and J: the joint rows, then one row per target */
                memset(Jt, 0, sizeof(double) * (size_t)m * n6);
                for (int r = 0; r < mj; ++r) {
                    F[r] = S.f[r];
                    for (int c = 0; c < n6; ++c) Jt[(size_t)r * n6 + c] = S.J[(size_t)r * n6 + c];
                }
                int r = mj;
                for (int j = R.j0; j < R.j1; ++j) {
                    if (isnan(target[j])) continue;
                    double Ja[6], Jb[6];
                    F[r] = joint_coordinate(&Bj, q_out, j, Ja, Jb) - target[j];
                    int la = local_body(B->joint_body[2 * j], R.b0), lb = local_body(B->joint_body[2 * j + 1], R.b0);
                    for (int k = 0; k < 6; ++k) {
                        if (la >= 0) Jt[(size_t)r * n6 + 6 * la + k] += Ja[k];
                        if (lb >= 0) Jt[(size_t)r * n6 + 6 * lb + k] += Jb[k];
                    }
                    ++r;
                }
                fn = inf_norm(m, F);
                if (fn <= tol || it >= max_iters) {
                    sys_free(&S);
                    break;
                }
                /* W J^T with W = M^-1, the base body's block zero */
                const int lbase = base ? local_body(base[w], R.b0) : -1;
                for (int i = 0; i < nb; ++i)
                    for (int a = 0; a < 6; ++a)
                        for (int k = 0; k < m; ++k) {
                            double s = 0.0;
                            if (i != lbase)
                                for (int c = 0; c < 6; ++c)
                                    s += S.Minv[36 * (size_t)i + 6 * a + c] * Jt[(size_t)k * n6 + 6 * i + c];
                            WJ[(size_t)(6 * i + a) * m + k] = s;
                        }
                double dmax = 0.0;
                for (int a = 0; a < m; ++a)
                    for (int b = 0; b < m; ++b) {
                        double s = 0.0;
                        for (int c = 0; c < n6; ++c) s += Jt[(size_t)a * n6 + c] * WJ[(size_t)c * m + b];
                        A[(size_t)a * m + b] = s;
                        if (a == b && s > dmax) dmax = s;
                    }
                const double mu = 1e-12 * (dmax > 0.0 ? dmax : 1.0);
                for (int a = 0; a < m; ++a) A[(size_t)a * m + a] += mu;
                if (orc_cholesky(m, A, L) != 0) {
                    sys_free(&S);
                    break;
                }
                chol_solve(m, L, F, y);
                for (int c = 0; c < n6; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < m; ++k) s += WJ[(size_t)c * m + k] * y[k];
                    Dl[c] = -s;
                }
                for (int i = 0; i < nb; ++i) {
                    double qn[7];
                    advance_pose(q_out + 7 * (size_t)(R.b0 + i), Dl + 6 * i, 1.0, qn);
                    for (int k = 0; k < 7; ++k) q_out[7 * (size_t)(R.b0 + i) + k] = qn[k];
                }
                ++it;
                sys_free(&S);
            }
            iters[w] = it;
            resid[w] = fn;
        }
        free(u0); free(Jt); free(F); free(WJ); free(A); free(L); free(y); free(Dl);
    }
    return err;
}
