"""FP64 CPU oracle for the constrained forward-dynamics step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the library.  It wraps the
plain C reference in ``kamx_oracle.c`` (built with gcc, no fast-math) through
ctypes; see that file for the equations it follows.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kamx_oracle.c")
LIB = os.path.join(HERE, "_kamx_oracle.so")

ROW_BILATERAL, ROW_LIMIT, ROW_NORMAL, ROW_TANGENT = 0, 1, 2, 3
OK, MAXITER, NONFINITE, FACTOR_FAIL = 0, 1, 2, 4


def build(force=True):
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over worlds)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-Wall", "-Wno-unused-function", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("gravity", C.c_double * 3), ("eta", C.c_double),
        ("rho_bil", C.c_double), ("rho_c", C.c_double), ("eps", C.c_double),
        ("max_iters", C.c_int32), ("fixed_iters", C.c_int32), ("accel", C.c_int32),
        ("restart_factor", C.c_double), ("precond", C.c_int32), ("baumgarte", C.c_double),
        ("warmstart", C.c_int32), ("replay", C.c_int32), ("log_stride", C.c_int32),
        ("integrator", C.c_int32), ("cr_iters", C.c_int32),
        ("adapt_ratio", C.c_double), ("adapt_factor", C.c_double), ("adapt_first", C.c_int32),
    ]


class _Batch(C.Structure):
    _fields_ = [
        ("n_worlds", C.c_int32), ("n_bodies", C.c_int32),
        ("body_world", C.c_void_p), ("mass", C.c_void_p), ("inertia", C.c_void_p),
        ("n_joints", C.c_int32), ("joint_type", C.c_void_p), ("joint_world", C.c_void_p),
        ("joint_body", C.c_void_p), ("joint_frame", C.c_void_p), ("joint_limit", C.c_void_p),
        ("n_contacts", C.c_int32), ("contact_world", C.c_void_p), ("contact_body", C.c_void_p),
        ("contact_point", C.c_void_p), ("contact_normal", C.c_void_p), ("contact_gap", C.c_void_p),
        ("contact_mu", C.c_void_p), ("joint_drive", C.c_void_p),
    ]


class _IO(C.Structure):
    _fields_ = [
        ("q", C.c_void_p), ("u", C.c_void_p), ("joint_torque", C.c_void_p), ("lambda_ws", C.c_void_p),
        ("q_out", C.c_void_p), ("u_out", C.c_void_p), ("lam", C.c_void_p), ("lambda_tilde", C.c_void_p),
        ("row_offset", C.c_void_p), ("iters", C.c_void_p), ("resid", C.c_void_p), ("status", C.c_void_p),
        ("restart_log", C.c_void_p),
    ]


@dataclass
class Params:
    """Solver parameters (Alg. 1 and Sec. 4.1)."""

    dt: float = 1e-3
    gravity: tuple = (0.0, 0.0, -9.81)
    eta: float = 1e-6
    rho_bil: float = 1e-6
    rho_c: float = 1.0
    eps: float = 1e-6
    max_iters: int = 2000
    fixed_iters: int = 0
    accel: int = 1
    restart_factor: float = 0.999
    precond: int = 1
    baumgarte: float = 0.2
    warmstart: int = 0
    integrator: int = 0  # 0 semi-implicit Euler, 1 Moreau-Jean midpoint (Sec. 3)
    cr_iters: int = 0    # 0 Cholesky; > 0 Conjugate Residual iterations per x-update (Sec. 5.1)
    # adaptive penalty on limit and contact rows (not in the paper; residual
    # balancing): 0 = off, else the ratio tau of r_d and r_p that triggers a
    # change by adapt_factor at iterations adapt_first * 2^j
    adapt_ratio: float = 0.0
    adapt_factor: float = 5.0
    adapt_first: int = 100

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)

    def _c(self, replay=0, log_stride=0):
        p = _Params()
        p.dt = self.dt
        for k in range(3):
            p.gravity[k] = self.gravity[k]
        p.eta, p.rho_bil, p.rho_c, p.eps = self.eta, self.rho_bil, self.rho_c, self.eps
        p.max_iters, p.fixed_iters, p.accel = self.max_iters, self.fixed_iters, self.accel
        p.restart_factor, p.precond, p.baumgarte = self.restart_factor, self.precond, self.baumgarte
        p.warmstart, p.replay, p.log_stride = self.warmstart, replay, log_stride
        p.integrator = self.integrator
        p.cr_iters = self.cr_iters
        p.adapt_ratio, p.adapt_factor, p.adapt_first = self.adapt_ratio, self.adapt_factor, self.adapt_first
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.POINTER(_Batch), C.POINTER(_Params), C.POINTER(_IO)]
        L.orc_row_offsets.argtypes = [C.POINTER(_Batch), C.c_void_p]
        L.orc_world_dims.argtypes = [C.POINTER(_Batch), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_world_system.restype = C.c_int
        L.orc_world_system.argtypes = [C.POINTER(_Batch), C.POINTER(_Params)] + [C.c_void_p] * 3 + [C.c_int] + [C.c_void_p] * 10
        L.orc_step_configuration.argtypes = [C.POINTER(_Batch), C.POINTER(_Params)] + [C.c_void_p] * 3
        L.orc_cr_solve.restype = C.c_int
        L.orc_cr_solve.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_fk.restype = C.c_int
        L.orc_fk.argtypes = [C.POINTER(_Batch), C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                             C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_joint_coordinate.restype = C.c_double
        L.orc_joint_coordinate.argtypes = [C.POINTER(_Batch), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        L.orc_project_block.argtypes = [C.c_int, C.c_double, C.c_void_p, C.c_void_p]
        L.orc_tangent_basis.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_solve_ncp.restype = C.c_int
        L.orc_solve_ncp.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(_Params),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int), C.c_void_p,
                                    C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


class _Keep:
    """Holds the contiguous arrays a C struct points into."""

    def __init__(self):
        self.items = []

    def __call__(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a


def _batch(scene, keep):
    b = _Batch()
    b.n_worlds = scene.n_worlds
    b.n_bodies = scene.n_bodies
    b.body_world = _p(keep(scene.body_world, np.int32))
    b.mass = _p(keep(scene.body_mass, np.float64))
    b.inertia = _p(keep(scene.body_inertia, np.float64))
    b.n_joints = scene.n_joints
    b.joint_type = _p(keep(scene.joint_type, np.int32))
    b.joint_world = _p(keep(scene.joint_world, np.int32))
    b.joint_body = _p(keep(scene.joint_body, np.int32))
    b.joint_frame = _p(keep(scene.joint_frame, np.float64))
    b.joint_limit = _p(keep(scene.joint_limit, np.float64))
    b.n_contacts = scene.n_contacts
    b.contact_world = _p(keep(scene.contact_world, np.int32))
    b.contact_body = _p(keep(scene.contact_body, np.int32))
    b.contact_point = _p(keep(scene.contact_point, np.float64))
    b.contact_normal = _p(keep(scene.contact_normal, np.float64))
    b.contact_gap = _p(keep(scene.contact_gap, np.float64))
    b.contact_mu = _p(keep(scene.contact_mu, np.float64))
    drive = getattr(scene, "joint_drive", None)
    b.joint_drive = _p(keep(drive, np.float64)) if drive is not None and drive.shape[0] == scene.n_joints and \
        scene.n_joints and np.any(drive[:, :4] != 0.0) else None
    return b


def row_offsets(scene):
    keep = _Keep()
    b = _batch(scene, keep)
    off = np.zeros(scene.n_worlds + 1, np.int64)
    lib().orc_row_offsets(C.byref(b), off.ctypes.data)
    return off


def step(scene, params: Params, q=None, u=None, joint_torque=None, lambda_ws=None,
         replay_log=None, log_iters=None):
    """One time step of every world.  Returns a dict with q, u (after the
    step), lam (impulses, physical units, per world rows concatenated),
    lam_tilde, row_offset, iters, resid [nw, 4], status and, when
    ``log_iters`` is given, the restart decisions [nw, log_iters]."""
    keep = _Keep()
    b = _batch(scene, keep)
    nw, nb = scene.n_worlds, scene.n_bodies
    off = row_offsets(scene)
    rows = int(off[-1])
    q = keep(scene.q if q is None else q, np.float64)
    u = keep(scene.u if u is None else u, np.float64)
    out = dict(
        q=np.zeros((nb, 7)), u=np.zeros((nb, 6)), lam=np.zeros(rows), lam_tilde=np.zeros(rows),
        row_offset=np.zeros(nw + 1, np.int64), iters=np.zeros(nw, np.int32), resid=np.zeros((nw, 4)),
        status=np.zeros(nw, np.int32),
    )
    stride = 0
    log = None
    replay = 0
    if replay_log is not None:
        log = keep(replay_log, np.uint8)
        stride = log.shape[1]
        replay = 1
    elif log_iters:
        stride = int(log_iters)
        log = np.zeros((nw, stride), np.uint8)
    io = _IO()
    io.q, io.u = _p(q), _p(u)
    io.joint_torque = _p(keep(joint_torque, np.float64)) if joint_torque is not None else None
    io.lambda_ws = _p(keep(lambda_ws, np.float64)) if lambda_ws is not None else None
    io.q_out, io.u_out = _p(out["q"]), _p(out["u"])
    io.lam, io.lambda_tilde = _p(out["lam"]), _p(out["lam_tilde"])
    io.row_offset = _p(out["row_offset"])
    io.iters, io.resid, io.status = _p(out["iters"]), _p(out["resid"]), _p(out["status"])
    io.restart_log = _p(log) if log is not None else None
    pp = params.replace(warmstart=1 if lambda_ws is not None else 0)._c(replay, stride)
    rc = lib().orc_step(C.byref(b), C.byref(pp), C.byref(io))
    if rc != 0:
        raise MemoryError("oracle step failed")
    if log is not None and not replay:
        out["restart_log"] = log
    return out


def world_dims(scene, w):
    keep = _Keep()
    b = _batch(scene, keep)
    nb, m = C.c_int(), C.c_int()
    lib().orc_world_dims(C.byref(b), w, C.byref(nb), C.byref(m))
    return nb.value, m.value


def world_system(scene, params: Params, w, q=None, u=None, joint_torque=None):
    """Assembled quantities of world ``w`` at the configuration of the step
    (the pre-step poses, or the half-step poses of the Moreau-Jean variant):
    J, f, vstar, kind, mu, Minv (nb x 6 x 6), uf, D (including R), vf and
    R (the diagonal regularisation of drive rows)."""
    keep = _Keep()
    b = _batch(scene, keep)
    nb, m = world_dims(scene, w)
    q = keep(scene.q if q is None else q, np.float64)
    u = keep(scene.u if u is None else u, np.float64)
    jt = keep(joint_torque, np.float64) if joint_torque is not None else None
    o = dict(J=np.zeros((m, 6 * nb)), f=np.zeros(m), vstar=np.zeros(m), kind=np.zeros(m, np.int32),
             mu=np.zeros(m), Minv=np.zeros((nb, 6, 6)), uf=np.zeros(6 * nb), D=np.zeros((m, m)),
             vf=np.zeros(m), R=np.zeros(m))
    pp = params._c()
    rc = lib().orc_world_system(C.byref(b), C.byref(pp), _p(q), _p(u), _p(jt) if jt is not None else None, w,
                                _p(o["J"]), _p(o["f"]), _p(o["vstar"]), _p(o["kind"]), _p(o["mu"]),
                                _p(o["Minv"]), _p(o["uf"]), _p(o["D"]), _p(o["vf"]), _p(o["R"]))
    if rc != 0:
        raise MemoryError("oracle world_system failed")
    return o


def step_configuration(scene, params: Params, q=None, u=None):
    """Poses at which the step evaluates constraints, forces and contacts:
    the pre-step poses (semi-implicit Euler) or the poses advanced by dt/2
    with the pre-step twists (Moreau-Jean midpoint)."""
    keep = _Keep()
    b = _batch(scene, keep)
    q = keep(scene.q if q is None else q, np.float64)
    u = keep(scene.u if u is None else u, np.float64)
    qm = np.zeros((scene.n_bodies, 7))
    pp = params._c()
    lib().orc_step_configuration(C.byref(b), C.byref(pp), _p(q), _p(u), _p(qm))
    return qm


def joint_coordinate(scene, q, j):
    keep = _Keep()
    b = _batch(scene, keep)
    q = keep(q, np.float64)
    Ja, Jb = np.zeros(6), np.zeros(6)
    c = lib().orc_joint_coordinate(C.byref(b), _p(q), j, _p(Ja), _p(Jb))
    return c, Ja, Jb


def cholesky(A):
    A = np.ascontiguousarray(A, np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    rc = lib().orc_cholesky(n, _p(A), _p(L))
    return L, rc


def project_block(kind, mu, w):
    w = np.ascontiguousarray(w, np.float64)
    o = np.zeros_like(w)
    lib().orc_project_block(kind, mu, _p(w), _p(o))
    return o


def tangent_basis(n):
    n = np.ascontiguousarray(n, np.float64)
    t1, t2 = np.zeros(3), np.zeros(3)
    lib().orc_tangent_basis(_p(n), _p(t1), _p(t2))
    return t1, t2


def solve_ncp(D, vf, kind, mu, params: Params, lambda_ws=None, log_iters=None):
    """PADMM on an explicit dual problem (Eq. 3): returns lambda, lambda_tilde,
    iterations, residuals, status and, when ``log_iters`` is given, the
    restart decision of each of the first log_iters iterations."""
    D = np.ascontiguousarray(D, np.float64)
    vf = np.ascontiguousarray(vf, np.float64)
    kind = np.ascontiguousarray(kind, np.int32)
    mu = np.ascontiguousarray(mu, np.float64)
    m = D.shape[0]
    lam, lt, res = np.zeros(m), np.zeros(m), np.zeros(4)
    it = C.c_int()
    ws = np.ascontiguousarray(lambda_ws, np.float64) if lambda_ws is not None else None
    pp = params.replace(warmstart=1 if ws is not None else 0)._c()
    log = np.zeros(max(int(log_iters or 0), params.fixed_iters or params.max_iters), np.uint8) if log_iters else None
    st = lib().orc_solve_ncp(m, _p(D), _p(vf), _p(kind), _p(mu), C.byref(pp), _p(ws) if ws is not None else None,
                             _p(lam), _p(lt), C.byref(it), _p(res), None, _p(log) if log is not None else None)
    out = dict(lam=lam, lam_tilde=lt, iters=it.value, resid=res, status=st)
    if log is not None:
        out["restart_log"] = log[:int(log_iters)]
    return out


def preconditioner(D, kind, enabled=True):
    """Sec. 4.1 Jacobi scales: D_ii^-1/2 per bilateral or limit row, one
    (trace of the 3 x 3 block / 3)^-1/2 per contact."""
    m = D.shape[0]
    p = np.ones(m)
    if not enabled:
        return p
    i = 0
    while i < m:
        if kind[i] == ROW_NORMAL:
            t = np.trace(D[i:i + 3, i:i + 3]) / 3.0
            p[i:i + 3] = 1.0 / np.sqrt(t) if t > 0 else 1.0
            i += 3
        else:
            p[i] = 1.0 / np.sqrt(D[i, i]) if D[i, i] > 0 else 1.0
            i += 1
    return p


def floor_report(scene, params: Params, w, q=None, u=None, joint_torque=None, rel_tol=1e-9):
    """Where lambda is not unique and where the dual residual has a floor
    (the paper's redundant loop rows, Sec. 3 and Sec. 4, are not discussed
    there; this is the reading used here).

    With J the world's constraint Jacobian, D~ = P J M^-1 J^T P and the
    bilateral rows B:

    * rank_J, rank_JB: numerical ranks of J and of its bilateral rows
      (singular values above rel_tol times the largest);
    * null_dim: m - rank_J, the dimension of the impulses that move no body
      (lambda is unique only when it is 0);
    * floor_inf: a lower bound on the infinity norm of the bilateral part of
      D~ lambda~ + v~_f for every lambda~.  Because J_B M^-1 J_C^T maps into
      the range of P_B J_B, the bilateral rows of D~ lambda~ stay in
      range(D~_BB) whatever the contact impulses; with n = P_N v~_f,B the
      component of the bilateral free velocity in null(D~_BB), every such
      vector w has <w, n> = |n|_2^2, hence |w|_inf >= |n|_2^2 / |n|_1.  The
      dual residual r_d of Alg. 1 cannot go below it (z = 0 on bilateral
      rows);
    * floor_2: |n|_2.

    Built on numpy's symmetric eigendecomposition of D~_BB (FP64)."""
    S = world_system(scene, params, w, q=q, u=u, joint_torque=joint_torque)
    J, D, vf, kind = S["J"], S["D"], S["vf"], S["kind"]
    m = J.shape[0]
    out = dict(m=m, rank_J=0, rank_JB=0, null_dim=0, floor_inf=0.0, floor_2=0.0)
    if m == 0:
        return out
    sv = np.linalg.svd(J, compute_uv=False)
    out["rank_J"] = int(np.sum(sv > rel_tol * sv.max())) if sv.size and sv.max() > 0 else 0
    out["null_dim"] = m - out["rank_J"]
    B = np.where(kind == ROW_BILATERAL)[0]
    if B.size == 0:
        return out
    svb = np.linalg.svd(J[B], compute_uv=False)
    out["rank_JB"] = int(np.sum(svb > rel_tol * svb.max())) if svb.max() > 0 else 0
    p = preconditioner(D, kind, params.precond)
    Dt = p[:, None] * D * p[None, :]
    DB = Dt[np.ix_(B, B)]
    ev, V = np.linalg.eigh(DB)
    N = V[:, ev <= rel_tol * max(ev.max(), 1e-300)]
    vt = (p * vf)[B]
    n = N @ (N.T @ vt) if N.shape[1] else np.zeros_like(vt)
    n2 = float(np.linalg.norm(n))
    out["floor_2"] = n2
    out["floor_inf"] = n2 * n2 / float(np.abs(n).sum()) if n2 > 0 else 0.0
    return out


def forward_kinematics(scene, targets, base=None, q=None, tol=1e-12, max_iters=100):
    """Sec. 6.3 forward kinematics by Gauss-Newton: poses that satisfy every
    joint constraint and put each joint with a finite entry of ``targets``
    [n_joints] at that coordinate, with body ``base[w]`` of each world held
    fixed (None: the scene's reset bodies; -1: none).  Returns (q [nb, 7],
    iterations [nw], |F|_inf [nw])."""
    keep = _Keep()
    b = _batch(scene, keep)
    q = keep(scene.q if q is None else q, np.float64)
    t = keep(targets, np.float64)
    if base is None:
        base = scene.reset_body if scene.reset_body.size == scene.n_worlds else np.full(scene.n_worlds, -1)
    bs = keep(base, np.int32)
    q_out = np.zeros((scene.n_bodies, 7))
    iters = np.zeros(scene.n_worlds, np.int32)
    res = np.zeros(scene.n_worlds)
    rc = lib().orc_fk(C.byref(b), _p(q), _p(t), _p(bs), float(tol), int(max_iters), _p(q_out), _p(iters), _p(res))
    if rc != 0:
        raise MemoryError("oracle forward kinematics failed")
    return q_out, iters, res


def set_threads(n):
    """Threads of the oracle's loops over worlds."""
    lib().orc_set_threads(int(n))


def cr_solve(A, b, n_iters, x0=None):
    """Conjugate Residual on the SPD system A x = b (Sec. 5.1's inner
    solver), n_iters iterations from x0 (default 0)."""
    A = np.ascontiguousarray(A, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(len(b)) if x0 is None else np.array(x0, np.float64)
    lib().orc_cr_solve(len(b), _p(A), _p(b), int(n_iters), _p(x))
    return x
