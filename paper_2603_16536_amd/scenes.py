"""Seeded synthetic scene generators (input side only).

This module builds batched maximal-coordinate worlds -- bodies, joints,
contact probe points and explicit contacts -- as plain numpy arrays in FP64.
It holds none of the solver's arithmetic: no Jacobians, no Delassus
operator, no cone projection, no time stepping.  The poses it writes are
assembled on the constraint manifold by elementary geometry (circle
intersection for the four-bar, parallelograms for the biped transmissions),
which is scene construction, not simulation.

Both the FP64 reference used by the tests and the HIP library consume the
arrays built here; nothing else is shared between them.

Conventions (a reading of Sec. 3, which leaves them open):
  * quaternions are stored (x, y, z, w);
  * twists are (v, w) with the angular velocity in the world frame;
  * a joint couples body ``a`` (always a real body) to body ``b``
    (``-1`` = the fixed world); each side carries a frame (position +
    quaternion) given in that body's frame (in the world frame for ``b=-1``);
    the joint axis is the frame's x axis;
  * a contact couples body ``a`` to body ``b`` (``-1`` = ground); its normal
    points from ``b`` towards ``a`` and a positive normal impulse pushes them
    apart.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

REVOLUTE = 0
PRISMATIC = 1

# ----------------------------------------------------------------------------
# small quaternion helpers for building poses (scene construction only)
# ----------------------------------------------------------------------------


def quat_axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    s = math.sin(0.5 * angle)
    return np.array([axis[0] * s, axis[1] * s, axis[2] * s, math.cos(0.5 * angle)])


def quat_mul(p, q):
    px, py, pz, pw = p
    qx, qy, qz, qw = q
    return np.array([
        pw * qx + px * qw + py * qz - pz * qy,
        pw * qy - px * qz + py * qw + pz * qx,
        pw * qz + px * qy - py * qx + pz * qw,
        pw * qw - px * qx - py * qy - pz * qz,
    ])


def quat_conj(q):
    return np.array([-q[0], -q[1], -q[2], q[3]])


def quat_to_mat(q):
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def quat_from_x_to(direction, up_hint=(0.0, 1.0, 0.0)):
    """Rotation whose x axis is ``direction`` and whose y axis is as close to
    ``up_hint`` as possible (a frame built by Gram-Schmidt)."""
    x = np.asarray(direction, np.float64)
    x = x / np.linalg.norm(x)
    y = np.asarray(up_hint, np.float64)
    y = y - x * np.dot(x, y)
    if np.linalg.norm(y) < 1e-9:
        y = np.array([0.0, 0.0, 1.0]) - x * x[2]
    y = y / np.linalg.norm(y)
    z = np.cross(x, y)
    return mat_to_quat(np.stack([x, y, z], axis=1))


def mat_to_quat(R):
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    if tr > 0:
        s = math.sqrt(tr + 1.0) * 2
        w = 0.25 * s
        x = (R[2, 1] - R[1, 2]) / s
        y = (R[0, 2] - R[2, 0]) / s
        z = (R[1, 0] - R[0, 1]) / s
    elif R[0, 0] > R[1, 1] and R[0, 0] > R[2, 2]:
        s = math.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        w = (R[2, 1] - R[1, 2]) / s
        x = 0.25 * s
        y = (R[0, 1] + R[1, 0]) / s
        z = (R[0, 2] + R[2, 0]) / s
    elif R[1, 1] > R[2, 2]:
        s = math.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        w = (R[0, 2] - R[2, 0]) / s
        x = (R[0, 1] + R[1, 0]) / s
        y = 0.25 * s
        z = (R[1, 2] + R[2, 1]) / s
    else:
        s = math.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        w = (R[1, 0] - R[0, 1]) / s
        x = (R[0, 2] + R[2, 0]) / s
        y = (R[1, 2] + R[2, 1]) / s
        z = 0.25 * s
    q = np.array([x, y, z, w])
    return q / np.linalg.norm(q)


def box_inertia(mass, sx, sy, sz):
    """Principal moments of a solid box with side lengths (sx, sy, sz)."""
    return np.array([
        mass * (sy * sy + sz * sz) / 12.0,
        mass * (sx * sx + sz * sz) / 12.0,
        mass * (sx * sx + sy * sy) / 12.0,
    ])


# ----------------------------------------------------------------------------
# the scene container
# ----------------------------------------------------------------------------


@dataclass
class Scene:
    """A batch of worlds.  Bodies, joints, probes and contacts are each
    sorted by world; indices into bodies are global (across the batch)."""

    n_worlds: int = 0
    body_world: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    body_mass: np.ndarray = field(default_factory=lambda: np.zeros(0))
    body_inertia: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    q: np.ndarray = field(default_factory=lambda: np.zeros((0, 7)))
    u: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    # box geometry per body (half extents, friction); zero rows: not a box
    body_box: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))

    joint_type: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    joint_world: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    joint_body: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    joint_frame: np.ndarray = field(default_factory=lambda: np.zeros((0, 14)))
    joint_limit: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    joint_actuated: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    # per-joint PD gains (kp, kd) toward the assembled coordinate; used when
    # the caller gives no global gains
    joint_pd: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    # implicit joint drives (kp, kd, damping, armature, ref) solved as
    # regularised rows; all zero: no drive row
    joint_drive: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))

    # contact probe points: body-frame points tested against the plane z = 0
    probe_world: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    probe_body: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    probe_point: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    probe_mu: np.ndarray = field(default_factory=lambda: np.zeros(0))

    # explicit contacts for single-step problems
    contact_world: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    contact_body: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    contact_point: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    contact_normal: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    contact_gap: np.ndarray = field(default_factory=lambda: np.zeros(0))
    contact_mu: np.ndarray = field(default_factory=lambda: np.zeros(0))
    contact_key: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    # per-world rollout extras: the body whose height triggers a reset
    reset_body: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    reset_height: float = -1.0e30

    gravity: tuple = (0.0, 0.0, -9.81)
    dt: float = 1e-3

    @property
    def n_bodies(self):
        return int(self.body_mass.shape[0])

    @property
    def n_joints(self):
        return int(self.joint_type.shape[0])

    @property
    def n_contacts(self):
        return int(self.contact_mu.shape[0])

    def offsets(self, world_ids):
        counts = np.bincount(world_ids, minlength=self.n_worlds)
        off = np.zeros(self.n_worlds + 1, np.int64)
        off[1:] = np.cumsum(counts)
        return off

    def body_offsets(self):
        return self.offsets(self.body_world)

    def joint_offsets(self):
        return self.offsets(self.joint_world)

    def contact_offsets(self):
        return self.offsets(self.contact_world)

    def probe_offsets(self):
        return self.offsets(self.probe_world)

    def subset(self, worlds):
        """A new scene made of the listed worlds (renumbered 0..k-1)."""
        worlds = np.asarray(worlds, np.int64)
        return concat([self._one(int(w)) for w in worlds], gravity=self.gravity, dt=self.dt,
                      reset_height=self.reset_height)

    def _one(self, w):
        bo, jo, co, po = self.body_offsets(), self.joint_offsets(), self.contact_offsets(), self.probe_offsets()
        b0, b1 = bo[w], bo[w + 1]
        s = Scene(n_worlds=1)
        s.body_world = np.zeros(b1 - b0, np.int32)
        s.body_mass = self.body_mass[b0:b1].copy()
        s.body_inertia = self.body_inertia[b0:b1].copy()
        s.q = self.q[b0:b1].copy()
        s.u = self.u[b0:b1].copy()
        s.body_box = _box_of(self)[b0:b1].copy()
        j0, j1 = jo[w], jo[w + 1]
        s.joint_type = self.joint_type[j0:j1].copy()
        s.joint_world = np.zeros(j1 - j0, np.int32)
        jb = self.joint_body[j0:j1].copy()
        s.joint_body = np.where(jb >= 0, jb - b0, -1).astype(np.int32)
        s.joint_frame = self.joint_frame[j0:j1].copy()
        s.joint_limit = self.joint_limit[j0:j1].copy()
        s.joint_actuated = self.joint_actuated[j0:j1].copy()
        s.joint_pd = _pd_of(self)[j0:j1].copy()
        s.joint_drive = _drive_of(self)[j0:j1].copy()
        p0, p1 = po[w], po[w + 1]
        s.probe_world = np.zeros(p1 - p0, np.int32)
        s.probe_body = (self.probe_body[p0:p1] - b0).astype(np.int32)
        s.probe_point = self.probe_point[p0:p1].copy()
        s.probe_mu = self.probe_mu[p0:p1].copy()
        c0, c1 = co[w], co[w + 1]
        s.contact_world = np.zeros(c1 - c0, np.int32)
        cb = self.contact_body[c0:c1].copy()
        s.contact_body = np.where(cb >= 0, cb - b0, -1).astype(np.int32)
        s.contact_point = self.contact_point[c0:c1].copy()
        s.contact_normal = self.contact_normal[c0:c1].copy()
        s.contact_gap = self.contact_gap[c0:c1].copy()
        s.contact_mu = self.contact_mu[c0:c1].copy()
        s.contact_key = self.contact_key[c0:c1].copy()
        if self.reset_body.size:
            rbw = int(self.reset_body[w])
            s.reset_body = np.array([rbw - b0 if rbw >= 0 else -1], np.int32)
        else:
            s.reset_body = np.zeros(0, np.int32)
        s.gravity = self.gravity
        s.dt = self.dt
        return s

    def replace(self, **kw):
        return dataclasses.replace(self, **kw)


def _box_of(s):
    return s.body_box if s.body_box.shape[0] == s.n_bodies else np.zeros((s.n_bodies, 4))


def _pd_of(s):
    return s.joint_pd if s.joint_pd.shape[0] == s.n_joints else np.zeros((s.n_joints, 2))


def _drive_of(s):
    return s.joint_drive if s.joint_drive.shape[0] == s.n_joints else np.zeros((s.n_joints, 5))


def concat(scenes, gravity=None, dt=None, reset_height=None):
    """Stack single- or multi-world scenes into one batch."""
    out = Scene(n_worlds=0)
    bw, bm, bi, q, u, bx = [], [], [], [], [], []
    jt, jw, jb, jf, jl, ja, jp, jd = [], [], [], [], [], [], [], []
    pw, pb, pp, pm = [], [], [], []
    cw, cb, cp, cn, cg, cm, ck = [], [], [], [], [], [], []
    rb = []
    nb = 0
    nw = 0
    for s in scenes:
        bw.append(s.body_world + nw)
        bm.append(s.body_mass)
        bi.append(s.body_inertia)
        q.append(s.q)
        u.append(s.u)
        bx.append(_box_of(s))
        jt.append(s.joint_type)
        jw.append(s.joint_world + nw)
        jb.append(np.where(s.joint_body >= 0, s.joint_body + nb, -1))
        jf.append(s.joint_frame)
        jl.append(s.joint_limit)
        ja.append(s.joint_actuated)
        jp.append(_pd_of(s))
        jd.append(_drive_of(s))
        pw.append(s.probe_world + nw)
        pb.append(s.probe_body + nb)
        pp.append(s.probe_point)
        pm.append(s.probe_mu)
        cw.append(s.contact_world + nw)
        cb.append(np.where(s.contact_body >= 0, s.contact_body + nb, -1))
        cp.append(s.contact_point)
        cn.append(s.contact_normal)
        cg.append(s.contact_gap)
        cm.append(s.contact_mu)
        ck.append(s.contact_key)
        if s.reset_body.size:
            rb.append(np.where(s.reset_body >= 0, s.reset_body + nb, -1))
        else:
            rb.append(np.full(s.n_worlds, -1, np.int32))
        nb += s.n_bodies
        nw += s.n_worlds
    out.n_worlds = nw
    out.body_world = np.concatenate(bw).astype(np.int32)
    out.body_mass = np.concatenate(bm)
    out.body_inertia = np.concatenate(bi).reshape(-1, 3)
    out.q = np.concatenate(q).reshape(-1, 7)
    out.u = np.concatenate(u).reshape(-1, 6)
    out.body_box = np.concatenate(bx).reshape(-1, 4)
    out.joint_type = np.concatenate(jt).astype(np.int32)
    out.joint_world = np.concatenate(jw).astype(np.int32)
    out.joint_body = np.concatenate(jb).reshape(-1, 2).astype(np.int32)
    out.joint_frame = np.concatenate(jf).reshape(-1, 14)
    out.joint_limit = np.concatenate(jl).reshape(-1, 2)
    out.joint_actuated = np.concatenate(ja).astype(np.int32)
    out.joint_pd = np.concatenate(jp).reshape(-1, 2)
    out.joint_drive = np.concatenate(jd).reshape(-1, 5)
    out.probe_world = np.concatenate(pw).astype(np.int32)
    out.probe_body = np.concatenate(pb).astype(np.int32)
    out.probe_point = np.concatenate(pp).reshape(-1, 3)
    out.probe_mu = np.concatenate(pm)
    out.contact_world = np.concatenate(cw).astype(np.int32)
    out.contact_body = np.concatenate(cb).reshape(-1, 2).astype(np.int32)
    out.contact_point = np.concatenate(cp).reshape(-1, 3)
    out.contact_normal = np.concatenate(cn).reshape(-1, 3)
    out.contact_gap = np.concatenate(cg)
    out.contact_mu = np.concatenate(cm)
    out.contact_key = np.concatenate(ck).astype(np.int32)
    out.reset_body = np.concatenate(rb).astype(np.int32)
    out.gravity = tuple(gravity if gravity is not None else scenes[0].gravity)
    out.dt = float(dt if dt is not None else scenes[0].dt)
    out.reset_height = float(reset_height if reset_height is not None else scenes[0].reset_height)
    return out


class _Builder:
    """Accumulates one world: bodies, joints, probes and contacts."""

    def __init__(self):
        self.mass, self.inertia, self.q, self.u = [], [], [], []
        self.jt, self.jb, self.jf, self.jl, self.ja, self.jp, self.jd = [], [], [], [], [], [], []
        self.pb, self.pp, self.pm = [], [], []
        self.cb, self.cp, self.cn, self.cg, self.cm, self.ck = [], [], [], [], [], []

    def body(self, mass, inertia, pos, quat, v=(0, 0, 0), w=(0, 0, 0)):
        self.mass.append(float(mass))
        self.inertia.append(np.asarray(inertia, np.float64))
        self.q.append(np.concatenate([np.asarray(pos, np.float64), np.asarray(quat, np.float64)]))
        self.u.append(np.concatenate([np.asarray(v, np.float64), np.asarray(w, np.float64)]))
        return len(self.mass) - 1

    def _local_frame(self, b, point_w, quat_w):
        if b < 0:
            return np.concatenate([np.asarray(point_w, np.float64), np.asarray(quat_w, np.float64)])
        r = self.q[b][:3]
        qb = self.q[b][3:]
        R = quat_to_mat(qb)
        p_local = R.T @ (np.asarray(point_w) - r)
        q_local = quat_mul(quat_conj(qb), quat_w)
        return np.concatenate([p_local, q_local])

    def joint(self, jtype, a, b, point_w, axis_w, limit=(np.nan, np.nan), actuated=0,
              point_b_w=None, pd=(0.0, 0.0), drive=(0.0, 0.0, 0.0, 0.0, 0.0)):
        """Joint whose frames coincide in the current (assembled) pose: both
        frames sit at ``point_w`` (``point_b_w`` for side b if given) with x
        along ``axis_w``."""
        qf = quat_from_x_to(axis_w)
        fa = self._local_frame(a, point_w, qf)
        fb = self._local_frame(b, point_w if point_b_w is None else point_b_w, qf)
        self.jt.append(jtype)
        self.jb.append((a, b))
        self.jf.append(np.concatenate([fa, fb]))
        self.jl.append(np.asarray(limit, np.float64))
        self.ja.append(int(actuated))
        self.jp.append(np.asarray(pd, np.float64))
        self.jd.append(np.asarray(drive, np.float64))
        return len(self.jt) - 1

    def probe(self, b, point_local, mu):
        self.pb.append(b)
        self.pp.append(np.asarray(point_local, np.float64))
        self.pm.append(float(mu))

    def contact(self, a, b, point_w, normal_w, gap, mu, key):
        n = np.asarray(normal_w, np.float64)
        self.cb.append((a, b))
        self.cp.append(np.asarray(point_w, np.float64))
        self.cn.append(n / np.linalg.norm(n))
        self.cg.append(float(gap))
        self.cm.append(float(mu))
        self.ck.append(int(key))

    def scene(self, dt, gravity=(0.0, 0.0, -9.81), reset_body=-1):
        s = Scene(n_worlds=1)
        nb = len(self.mass)
        s.body_world = np.zeros(nb, np.int32)
        s.body_mass = np.array(self.mass)
        s.body_inertia = np.array(self.inertia).reshape(-1, 3)
        s.q = np.array(self.q).reshape(-1, 7)
        s.u = np.array(self.u).reshape(-1, 6)
        nj = len(self.jt)
        s.joint_type = np.array(self.jt, np.int32)
        s.joint_world = np.zeros(nj, np.int32)
        s.joint_body = np.array(self.jb, np.int32).reshape(-1, 2)
        s.joint_frame = np.array(self.jf).reshape(-1, 14)
        s.joint_limit = np.array(self.jl).reshape(-1, 2)
        s.joint_actuated = np.array(self.ja, np.int32)
        s.joint_pd = np.array(self.jp).reshape(-1, 2)
        s.joint_drive = np.array(self.jd).reshape(-1, 5)
        npb = len(self.pb)
        s.probe_world = np.zeros(npb, np.int32)
        s.probe_body = np.array(self.pb, np.int32)
        s.probe_point = np.array(self.pp).reshape(-1, 3)
        s.probe_mu = np.array(self.pm)
        nc = len(self.cb)
        s.contact_world = np.zeros(nc, np.int32)
        s.contact_body = np.array(self.cb, np.int32).reshape(-1, 2)
        s.contact_point = np.array(self.cp).reshape(-1, 3)
        s.contact_normal = np.array(self.cn).reshape(-1, 3)
        s.contact_gap = np.array(self.cg)
        s.contact_mu = np.array(self.cm)
        s.contact_key = np.array(self.ck, np.int32)
        s.reset_body = np.array([reset_body], np.int32)
        s.dt = dt
        s.gravity = tuple(gravity)
        return s


def _rod_body(B, p0, p1, mass, width=0.02, v=(0, 0, 0), w=(0, 0, 0)):
    """A slender box between points p0 and p1 (body x axis along the rod)."""
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    L = float(np.linalg.norm(p1 - p0))
    q = quat_from_x_to(p1 - p0, up_hint=(0.0, 1.0, 0.0))
    return B.body(mass, box_inertia(mass, L, width, width), 0.5 * (p0 + p1), q, v, w)


def add_ground_contacts_from_probes(B, gap_max=np.inf):
    """Explicit contacts for the current poses: every probe point whose
    height above z = 0 is below ``gap_max`` becomes a contact with normal +z
    against the ground."""
    for k, (b, pl, mu) in enumerate(zip(B.pb, B.pp, B.pm)):
        R = quat_to_mat(B.q[b][3:])
        pw = B.q[b][:3] + R @ pl
        if pw[2] < gap_max:
            B.contact(b, -1, pw, (0.0, 0.0, 1.0), pw[2], mu, k)


# ----------------------------------------------------------------------------
# worlds
# ----------------------------------------------------------------------------


def pendulum(length=0.5, mass=1.0, theta0=0.3, omega0=0.0, dt=1e-3, width=0.02):
    """One slender rod hinged to the world at the origin about world y.
    ``theta0`` is the angle from the downward vertical (positive towards +x)."""
    B = _Builder()
    d = np.array([math.sin(theta0), 0.0, -math.cos(theta0)])
    p1 = length * d
    # angular velocity about world y; with d = (sin, 0, -cos), rotating by +omega
    # about -y increases theta, so w = (0, -omega0, 0)
    wv = np.array([0.0, -omega0, 0.0])
    com = 0.5 * p1
    v = np.cross(wv, com)
    rod = _rod_body(B, np.zeros(3), p1, mass, width, v=v, w=wv)
    B.joint(REVOLUTE, rod, -1, np.zeros(3), (0.0, 1.0, 0.0))
    return B.scene(dt)


def box_on_incline(theta, mu, mass=1.0, size=(0.2, 0.2, 0.05), dt=1e-3, g=9.81):
    """A flat box resting on a plane through the origin tilted by ``theta``
    about world y (downhill towards +x); four bottom corners in contact."""
    B = _Builder()
    qp = quat_axis_angle((0.0, 1.0, 0.0), theta)  # plane frame
    Rp = quat_to_mat(qp)
    n = Rp @ np.array([0.0, 0.0, 1.0])
    sx, sy, sz = size
    com = n * (0.5 * sz)
    box = B.body(mass, box_inertia(mass, sx, sy, sz), com, qp)
    k = 0
    for ix in (-1, 1):
        for iy in (-1, 1):
            pl = np.array([0.5 * sx * ix, 0.5 * sy * iy, -0.5 * sz])
            B.probe(box, pl, mu)
            pw = com + Rp @ pl
            B.contact(box, -1, pw, n, 0.0, mu, k)
            k += 1
    return B.scene(dt, gravity=(0.0, 0.0, -g))


def fourbar_geometry(rng):
    """Rejection-sample a planar four-bar (ground d, crank a, coupler b,
    rocker c) that assembles at crank angle th2 with a healthy transmission
    angle; returns the link lengths, th2 and the joint points in the x-z
    plane (pivot A at the origin, pivot D at (d, 0))."""
    while True:
        a, b, c, d = rng.uniform(0.05, 0.3, 4)
        th2 = 0.5 * math.pi + rng.uniform(-0.3, 0.3)
        P = np.array([a * math.cos(th2), a * math.sin(th2)])
        D = np.array([d, 0.0])
        e = D - P
        dist = float(np.linalg.norm(e))
        if not (abs(b - c) + 0.01 < dist < b + c - 0.01):
            continue
        # circle-circle intersection: Q with |Q - P| = b, |Q - D| = c
        x = (dist * dist + b * b - c * c) / (2 * dist)
        h = math.sqrt(max(b * b - x * x, 0.0))
        ex = e / dist
        ey = np.array([-ex[1], ex[0]])
        Q = P + x * ex + h * ey  # the "open" branch (left of P->D)
        # transmission angle between coupler and rocker
        u1 = (Q - P) / b
        u2 = (Q - D) / c
        s = abs(u1[0] * u2[1] - u1[1] * u2[0])
        if s < 0.3:
            continue
        return dict(a=a, b=b, c=c, d=d, th2=th2, P=P, Q=Q, D=D)


def fourbar_world(rng, with_box=True, dt=1e-3, origin=(0.0, 0.0, 0.6), box_mu=0.8):
    """Four-bar linkage in the vertical x-z plane plus (optionally) a 0.1 m
    cube sliding on the ground with four corner contacts.  The ground link is
    the world; links 1-3 are dynamic boxes with a 0.02 m square section."""
    geo = fourbar_geometry(rng)
    O = np.asarray(origin, np.float64)

    def w3(p2):
        return O + np.array([p2[0], 0.0, p2[1]])

    A, P, Q, D = w3(np.zeros(2)), w3(geo["P"]), w3(geo["Q"]), w3(geo["D"])
    masses = rng.uniform(0.1, 2.0, 3)
    B = _Builder()
    crank = _rod_body(B, A, P, masses[0])
    coupler = _rod_body(B, P, Q, masses[1])
    rocker = _rod_body(B, D, Q, masses[2])
    y = (0.0, 1.0, 0.0)
    B.joint(REVOLUTE, crank, -1, A, y, actuated=1)
    B.joint(REVOLUTE, coupler, crank, P, y)
    B.joint(REVOLUTE, rocker, coupler, Q, y)
    B.joint(REVOLUTE, rocker, -1, D, y)
    if with_box:
        vx = rng.uniform(-0.5, 0.5)
        c = np.array([0.0, 1.0, 0.05])
        box = B.body(1.0, box_inertia(1.0, 0.1, 0.1, 0.1), c, np.array([0, 0, 0, 1.0]), v=(vx, 0, 0))
        for ix in (-1, 1):
            for iy in (-1, 1):
                B.probe(box, (0.05 * ix, 0.05 * iy, -0.05), box_mu)
        add_ground_contacts_from_probes(B, gap_max=1e-2)
    s = B.scene(dt)
    s.meta = geo  # type: ignore[attr-defined]
    return s


def free_fourbar_world(rng, dt=1e-3, origin=(0.0, 0.0, 0.6), v_scale=0.3, w_scale=1.0):
    """Four dynamic links (the four-bar's ground link as a body too) joined
    in one closed loop, attached to nothing, with random twists (not
    consistent with the joints) and no gravity: every constraint impulse is
    internal to the mechanism."""
    geo = fourbar_geometry(rng)
    O = np.asarray(origin, np.float64)

    def w3(p2):
        return O + np.array([p2[0], 0.0, p2[1]])

    A, P, Q, D = w3(np.zeros(2)), w3(geo["P"]), w3(geo["Q"]), w3(geo["D"])
    masses = rng.uniform(0.1, 2.0, 4)
    B = _Builder()
    ground = _rod_body(B, A, D, masses[3])
    crank = _rod_body(B, A, P, masses[0])
    coupler = _rod_body(B, P, Q, masses[1])
    rocker = _rod_body(B, D, Q, masses[2])
    y = (0.0, 1.0, 0.0)
    B.joint(REVOLUTE, crank, ground, A, y)
    B.joint(REVOLUTE, coupler, crank, P, y)
    B.joint(REVOLUTE, rocker, coupler, Q, y)
    B.joint(REVOLUTE, rocker, ground, D, y)
    s = B.scene(dt, gravity=(0.0, 0.0, 0.0))
    s.u = np.concatenate([rng.normal(0.0, v_scale, (s.n_bodies, 3)), rng.normal(0.0, w_scale, (s.n_bodies, 3))], axis=1)
    return s


def free_fourbar_batch(n_worlds, seed=1006, dt=1e-3):
    rng = np.random.default_rng(seed)
    return concat([free_fourbar_world(rng, dt) for _ in range(n_worlds)])


def fourbar_batch(n_worlds, seed=1001, with_box=True, dt=1e-3):
    rng = np.random.default_rng(seed)
    return concat([fourbar_world(rng, with_box, dt) for _ in range(n_worlds)])


# --- biped ------------------------------------------------------------------

BIPED_FOOT = (0.20, 0.10, 0.04)


BIPED_PD = (15.0, 0.6)  # N m / rad, N m s / rad: the DR Legs gains of the paper's RL setup (Sec. 6.3)


def biped_world(rng, dt=2e-3, mu=None, link_masses=None, sole_probes=4):
    """A 31-body biped: pelvis + 2 legs x (hip-yaw, hip-roll, thigh, shin,
    foot) + 2 legs x 5 crank-rod parallelogram transmissions (2 bodies and 3
    revolute joints each).  40 revolute joints (200 bilateral rows), four
    sole probe points per foot (8 contacts, 24 rows).  Stands on z = 0 with
    straight legs at rest; exactly on the constraint manifold.  The ten chain
    joints (hip yaw, roll, pitch, knee, ankle of each leg) are actuated; the
    3-30 g transmission links are passive.  sole_probes = 2 keeps only the
    heel and toe of each sole's centre line (12 contact rows instead of 24,
    which leaves room in the 224-row bucket for ten drive rows)."""
    if mu is None:
        mu = rng.uniform(0.5, 1.0)
    if link_masses is None:
        link_masses = rng.uniform(0.003, 0.030, 20)
    fx, fy, fz = BIPED_FOOT
    ankle_z = fz + 0.015
    knee_z = ankle_z + 0.25
    hip_z = knee_z + 0.25
    H = hip_z + 0.12
    B = _Builder()
    ident = np.array([0.0, 0.0, 0.0, 1.0])
    pelvis = B.body(3.0, box_inertia(3.0, 0.20, 0.30, 0.12), (0.0, 0.0, H), ident)
    xa, ya, za = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)
    lm = iter(link_masses)
    for side in (1.0, -1.0):
        yl = 0.09 * side
        hy = B.body(0.5, box_inertia(0.5, 0.06, 0.06, 0.04), (0.0, yl, H - 0.05), ident)
        B.joint(REVOLUTE, hy, pelvis, (0.0, yl, H - 0.03), za, actuated=1, pd=BIPED_PD)
        hr = B.body(0.5, box_inertia(0.5, 0.06, 0.06, 0.04), (0.0, yl, H - 0.10), ident)
        B.joint(REVOLUTE, hr, hy, (0.0, yl, H - 0.08), xa, actuated=1, pd=BIPED_PD)
        Hp = np.array([0.0, yl, hip_z])
        Kn = np.array([0.0, yl, knee_z])
        An = np.array([0.0, yl, ankle_z])
        thigh = _rod_body(B, Hp, Kn, 1.2, width=0.06)
        B.joint(REVOLUTE, thigh, hr, Hp, ya, actuated=1, pd=BIPED_PD)
        shin = _rod_body(B, Kn, An, 0.8, width=0.05)
        B.joint(REVOLUTE, shin, thigh, Kn, ya, actuated=1, pd=BIPED_PD)
        fc = np.array([0.02, yl, 0.5 * fz])  # sole on z = 0
        foot = B.body(0.6, box_inertia(0.6, fx, fy, fz), fc, ident)
        B.joint(REVOLUTE, foot, shin, An, ya, actuated=1, pd=BIPED_PD)
        for ix in (-1, 1):
            for iy in ((-1, 1) if sole_probes == 4 else (0,)):
                B.probe(foot, (0.5 * fx * ix, 0.5 * fy * iy, -0.5 * fz), mu)
        # parallelogram transmissions: (parent, child, joint point, delta, crank)
        loops = [
            (hr, thigh, Hp, (-0.04, 0.0, 0.0), (0.0, 0.0, -0.06), 0),
            (thigh, shin, Kn, (0.035, 0.0, 0.0), (0.0, 0.0, -0.07), 0),
            (thigh, shin, Kn, (-0.035, 0.0, 0.02), (0.01, 0.0, -0.09), 0),
            (shin, foot, An, (0.03, 0.0, 0.04), (0.05, 0.0, 0.0), 0),
            (shin, foot, An, (-0.03, 0.0, 0.05), (-0.04, 0.0, -0.01), 0),
        ]
        for li, (par, chi, K, dl, cr, act) in enumerate(loops):
            dy = np.array([0.0, 0.012 * side * (li + 1), 0.0])
            Kp = K + np.asarray(dl) + dy
            Kc = Kp + np.asarray(cr)
            Kr = K + np.asarray(cr) + dy
            crank = _rod_body(B, Kp, Kc, next(lm), width=0.01)
            rod = _rod_body(B, Kc, Kr, next(lm), width=0.01)
            B.joint(REVOLUTE, crank, par, Kp, ya, actuated=act)
            B.joint(REVOLUTE, rod, crank, Kc, ya)
            B.joint(REVOLUTE, rod, chi, Kr, ya)
    add_ground_contacts_from_probes(B)
    return B.scene(dt, reset_body=pelvis)


BIPED_ARMATURE = 5e-4  # kg m^2: reflected rotor inertia of a transmission drive


def with_drives(scene, mode="implicit", pd=BIPED_PD, armature=BIPED_ARMATURE, damping=0.01):
    """The biped with joint drives as regularised rows (Sec. 3 implicit PD,
    armature and viscous damping) instead of explicit PD:

    * "implicit": the ten actuated chain joints keep their gains, solved as
      implicit PD rows toward the assembled pose;
    * "transmission": the hip yaw and roll joints keep their explicit PD,
      the hip pitch, knee and ankle chain joints are passive, and the ten
      crank joints of the parallelogram transmissions are actuated instead
      (implicit PD, rotor armature and damping; noise acts on them), as the
      paper's DR Legs drives its legs through the linkages (Sec. 6.1).

    Either adds ten drive rows: with the 200 joint rows the scene must come
    from biped_batch(..., sole_probes=2) to fit the 224-row bucket."""
    s = scene.replace(joint_drive=np.zeros((scene.n_joints, 5)), joint_actuated=scene.joint_actuated.copy(),
                      joint_pd=scene.joint_pd.copy())
    jo = scene.joint_offsets()
    for w in range(scene.n_worlds):
        js = range(jo[w], jo[w + 1])
        chain = [j for j in js if scene.joint_actuated[j]]
        if mode == "implicit":
            for j in chain:
                s.joint_drive[j] = (pd[0], pd[1], 0.0, 0.0, 0.0)
                s.joint_pd[j] = (0.0, 0.0)
            continue
        # per leg: 5 chain joints then 5 loops of 3 joints (crank, rod-crank, rod-child)
        local = [j - jo[w] for j in js]
        for leg in range(2):
            base = 20 * leg
            for k in (2, 3, 4):  # hip pitch, knee, ankle: driven through the linkages
                s.joint_actuated[jo[w] + base + k] = 0
                s.joint_pd[jo[w] + base + k] = (0.0, 0.0)
            for li in range(5):
                crank = jo[w] + base + 5 + 3 * li
                s.joint_actuated[crank] = 1
                s.joint_drive[crank] = (pd[0], pd[1], damping, armature, 0.0)
        assert len(local) == 40
    return s


def biped_batch(n_worlds, seed=1002, dt=2e-3, sole_probes=4):
    """``n_worlds`` identical bipeds (transmission masses drawn once from
    the seed) with a per-world friction coefficient mu ~ U[0.5, 1.0]."""
    rng = np.random.default_rng(seed)
    link_masses = rng.uniform(0.003, 0.030, 20)
    mus = rng.uniform(0.5, 1.0, n_worlds)
    one = biped_world(rng, dt, mu=0.75, link_masses=link_masses, sole_probes=sole_probes)
    s = concat([one] * n_worlds, reset_height=0.2)
    # per-world friction
    s.probe_mu = np.repeat(mus, 2 * sole_probes)
    s.contact_mu = np.repeat(mus, 2 * sole_probes)
    return s


FIGURE_PD = {"base": (400.0, 8.0), "leg": (200.0, 4.0), "torso": (300.0, 6.0), "head": (20.0, 0.4),
             "arm": (100.0, 2.0), "finger": (0.2, 0.004)}  # N m / rad, N m s / rad


def axis_inertia(mass, inertia, pose, point, axis):
    """Moment of inertia of one body about the line through ``point`` along
    the unit ``axis`` (world frame): the principal inertia rotated to the
    world, plus the parallel-axis term of the centre of mass."""
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    R = quat_to_mat(np.asarray(pose[3:], np.float64))
    Iw = R @ np.diag(np.asarray(inertia, np.float64)) @ R.T
    r = np.asarray(pose[:3], np.float64) - np.asarray(point, np.float64)
    return float(a @ Iw @ a + mass * (r @ r - (a @ r) ** 2))


def explicit_pd_gains(nominal, mass, inertia, pose, point, axis, dt):
    """Gains of an explicit PD torque on a joint, capped so that it stays
    stable at step dt: an explicit spring-damper on an inertia I advances
    omega by -(kd dt / I) omega - (kp dt^2 / I) theta per step, which is
    stable for kd dt / I < 2 and kp dt^2 / I small; the caps are
    kd dt / I <= 0.5 and kp dt^2 / I <= 0.1 with I the child body's own
    inertia about the joint axis (the subtree moved by the joint only adds
    to it)."""
    kp, kd = nominal
    I = axis_inertia(mass, inertia, pose, point, axis)
    return min(kp, 0.1 * I / (dt * dt)), min(kd, 0.5 * I / dt)


def _perp_pair(a):
    """Two unit vectors completing the unit axis a to a right-handed frame."""
    a = np.asarray(a, np.float64)
    h = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    d1 = np.cross(a, h)
    d1 /= np.linalg.norm(d1)
    return d1, np.cross(a, d1)


def figure_world(rng, dt=2e-3, link_masses=None):
    """A figure fixed to the ground with the size of the paper's largest
    system (Tab. 1: 151 bodies, 27 actuated and 169 passive joints, 45
    independent loops): a 61-body tree -- base on a yaw joint to the world,
    two legs (hip yaw, roll, pitch, knee, ankle), torso (waist pitch, chest
    roll, yaw), head (neck pitch, yaw, jaw), two arms (shoulder pitch, roll,
    upper-arm yaw, elbow, forearm roll, wrist, hand) and five three-phalanx
    fingers per hand -- whose hip-pitch, knee, ankle, waist, chest,
    chest-yaw, neck, jaw, elbow and wrist joints and every finger joint are each driven
    through a crank-rod parallelogram (2 bodies, 3 revolute joints: 45
    loops).  196 revolute joints (980 bilateral rows), no contacts.  27 tree
    joints (base, legs, torso, head, arms except forearm roll and hand) are
    actuated: explicit PD toward the assembled pose plus noise; the other
    34 tree joints (forearm roll, hand, fingers) are passive spring-damper
    couplings toward the assembled pose, solved implicitly as drive rows
    (Sec. 3), which makes 1014 rows.
    The 3-30 g transmission links against the 8 kg base give a mass ratio
    of about 3e3.  Exactly on the constraint manifold."""
    if link_masses is None:
        link_masses = rng.uniform(0.003, 0.030, 90)
    lm = iter(link_masses)
    B = _Builder()
    ident = np.array([0.0, 0.0, 0.0, 1.0])
    xa, ya, za = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0])
    H = 1.35
    tree = []  # (parent, child, point, axis, kind, actuated, looped)

    def link(parent, p0, p1, mass, width, axis, kind, act, looped, joint_point=None):
        b = _rod_body(B, p0, p1, mass, width=width)
        K = np.asarray(p0 if joint_point is None else joint_point, np.float64)
        if act:
            B.joint(REVOLUTE, b, parent, K, axis, actuated=1,
                    pd=explicit_pd_gains(FIGURE_PD[kind], B.mass[b], B.inertia[b], B.q[b], K, axis, dt))
        else:  # a passive spring-damper coupling, solved as an implicit drive row
            kp, kd = FIGURE_PD[kind]
            B.joint(REVOLUTE, b, parent, K, axis, drive=(kp, kd, 0.0, 0.0, 0.0))
        tree.append((parent, b, K, np.asarray(axis, np.float64), looped))
        return b

    base = B.body(8.0, box_inertia(8.0, 0.30, 0.22, 0.16), (0.0, 0.0, H), ident)
    B.joint(REVOLUTE, base, -1, (0.0, 0.0, H - 0.08), za, actuated=1,
            pd=explicit_pd_gains(FIGURE_PD["base"], B.mass[base], B.inertia[base], B.q[base], (0.0, 0.0, H - 0.08),
                                 za, dt))
    # legs
    for sd in (1.0, -1.0):
        y = 0.1 * sd
        hy = link(base, (0, y, H - 0.08), (0, y, H - 0.14), 0.8, 0.06, za, "leg", 1, False)
        hr = link(hy, (0, y, H - 0.14), (0, y, H - 0.20), 0.8, 0.06, xa, "leg", 1, False)
        th = link(hr, (0, y, H - 0.20), (0, y, H - 0.62), 3.0, 0.08, ya, "leg", 1, True)
        sh = link(th, (0, y, H - 0.62), (0, y, H - 1.02), 2.0, 0.06, ya, "leg", 1, True)
        link(sh, (0, y, H - 1.02), (0.12, y, H - 1.08), 0.8, 0.06, ya, "leg", 1, True)
    # torso and head
    wa = link(base, (0, 0, H + 0.08), (0, 0, H + 0.25), 4.0, 0.2, ya, "torso", 1, True)
    ch = link(wa, (0, 0, H + 0.25), (0, 0, H + 0.45), 5.0, 0.25, xa, "torso", 1, True)
    uc = link(ch, (0, 0, H + 0.45), (0, 0, H + 0.60), 3.0, 0.25, za, "torso", 1, True)
    nk = link(uc, (0, 0, H + 0.60), (0, 0, H + 0.70), 0.6, 0.06, ya, "head", 1, True)
    hd = link(nk, (0, 0, H + 0.70), (0, 0, H + 0.88), 2.5, 0.16, za, "head", 1, False)
    link(hd, (0.05, 0, H + 0.75), (0.12, 0, H + 0.72), 0.3, 0.05, ya, "head", 1, True)
    # arms and hands (T-pose along +-y)
    for sd in (1.0, -1.0):
        y0 = 0.16 * sd
        z = H + 0.55
        e = np.array([0.0, sd, 0.0])
        p = lambda d: np.array([0.0, y0, z]) + d * e
        s1 = link(uc, p(0.0), p(0.05), 0.6, 0.07, ya, "arm", 1, False)
        s2 = link(s1, p(0.05), p(0.10), 0.6, 0.07, xa, "arm", 1, False)
        ua = link(s2, p(0.10), p(0.38), 2.0, 0.07, e, "arm", 1, False)
        fa = link(ua, p(0.38), p(0.58), 1.2, 0.06, za, "arm", 1, True)
        fr = link(fa, p(0.58), p(0.64), 0.4, 0.05, e, "arm", 0, False)
        wr = link(fr, p(0.64), p(0.68), 0.3, 0.05, za, "arm", 1, True)
        hand = link(wr, p(0.68), p(0.78), 0.4, 0.06, xa, "arm", 0, False)
        for f in range(5):
            off = np.array([0.0, 0.0, -0.03 + 0.015 * f])
            q0 = p(0.78) + off
            prev = hand
            for ph in range(3):
                a0 = q0 + (0.035 * ph) * e
                a1 = q0 + (0.035 * (ph + 1)) * e
                prev = link(prev, a0, a1, 0.03 - 0.006 * ph, 0.012, xa, "finger", 0, True)
    assert len(B.mass) == 61 and len(B.jt) == 61, (len(B.mass), len(B.jt))
    # crank-rod parallelograms across the looped tree joints
    loops = [t for t in tree if t[4]]
    assert len(loops) == 45, len(loops)
    for li, (par, chi, K, a, _) in enumerate(loops):
        d1, d2 = _perp_pair(a)
        s_ = 0.012 * (1 if li % 2 == 0 else -1)
        Kp = K + 0.025 * d1 + s_ * a
        Kc = Kp + 0.035 * d2
        Kr = K + 0.035 * d2 + s_ * a
        crank = _rod_body(B, Kp, Kc, next(lm), width=0.008)
        rod = _rod_body(B, Kc, Kr, next(lm), width=0.008)
        B.joint(REVOLUTE, crank, par, Kp, a)
        B.joint(REVOLUTE, rod, crank, Kc, a)
        B.joint(REVOLUTE, rod, chi, Kr, a)
    return B.scene(dt, reset_body=-1)


def figure_batch(n_worlds, seed=1007, dt=2e-3):
    """n_worlds identical fixed figures (transmission masses drawn once)."""
    rng = np.random.default_rng(seed)
    one = figure_world(rng, dt)
    return concat([one] * n_worlds)


def _circle_intersection(c0, r0, c1, r1, side):
    """A point at distance r0 from c0 and r1 from c1 in the x-z plane
    (y of c0), on the side of the c0->c1 line given by the sign of side."""
    c0 = np.asarray(c0, np.float64)
    c1 = np.asarray(c1, np.float64)
    d = c1 - c0
    L = float(np.hypot(d[0], d[2]))
    if not (abs(r0 - r1) < L < r0 + r1):
        raise ValueError("circles do not intersect")
    a = (r0 * r0 - r1 * r1 + L * L) / (2 * L)
    h = np.sqrt(r0 * r0 - a * a)
    ex = d / L
    ez = np.array([-ex[2], 0.0, ex[0]])  # in-plane normal
    return c0 + a * ex + np.sign(side) * h * ez


def excavator_world(rng, dt=2e-3):
    """A 12-body hydraulic excavator: cab on a swing revolute to the world;
    boom, stick and bucket on revolute pins; three hydraulic cylinders
    (barrel and rod on revolute pins, joined by a prismatic joint with a
    stroke limit); a bucket linkage of two links closing a four-bar with the
    stick and bucket, the bucket cylinder's rod pinned at the links' common
    pin.  16 joints (13 revolute, 3 prismatic), 4 kinematic loops, 80
    bilateral rows + 3 stroke-limit rows.  Masses from 5000 kg (cab) down to
    0.5 kg (linkage links): mass ratio 1e4.  Geometry jittered by a few per
    cent per world, assembled exactly (circle intersection for the bucket
    four-bar).  The swing and the three cylinders hold their assembled
    coordinates with PD gains."""
    j = lambda: 1.0 + rng.uniform(-0.04, 0.04)
    ident = np.array([0.0, 0.0, 0.0, 1.0])
    ya, za = (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)
    B = _Builder()
    cab = B.body(5000.0, box_inertia(5000.0, 3.0, 2.5, 1.5), (0.0, 0.0, 1.55), ident)
    B.joint(REVOLUTE, cab, -1, (0.0, 0.0, 0.8), za, actuated=1, pd=(2.0e5, 2.0e4))
    P0 = np.array([0.8 * j(), 0.0, 2.0])           # boom foot pin (on the cab)
    P1 = P0 + np.array([3.2 * j(), 0.0, 1.6 * j()])  # boom tip / stick pin
    P2 = P1 + np.array([1.4 * j(), 0.0, -2.4 * j()])  # stick tip / bucket pin
    P3 = P2 + np.array([0.35, 0.0, -0.65 * j()])      # bucket teeth
    boom = _rod_body(B, P0, P1, 800.0, width=0.5)
    stick = _rod_body(B, P1, P2, 400.0, width=0.35)
    bucket = _rod_body(B, P2, P3, 300.0, width=0.8)
    B.joint(REVOLUTE, boom, cab, P0, ya)
    B.joint(REVOLUTE, stick, boom, P1, ya)
    B.joint(REVOLUTE, bucket, stick, P2, ya)
    cyls = []

    def cylinder(body0, a, body1, b, m_barrel, m_rod, stroke=0.35):
        a = np.asarray(a, np.float64)
        b = np.asarray(b, np.float64)
        mid = 0.5 * (a + b)
        barrel = _rod_body(B, a, mid + 0.1 * (b - a), m_barrel, width=0.18)
        rod = _rod_body(B, mid - 0.1 * (b - a), b, m_rod, width=0.10)
        B.joint(REVOLUTE, barrel, body0, a, ya)
        B.joint(REVOLUTE, rod, body1, b, ya)
        # slide coordinate measured from the assembled stroke
        cyls.append(B.joint(PRISMATIC, rod, barrel, mid, b - a, limit=(-stroke, stroke), actuated=1,
                            pd=(4.0e6, 2.0e5)))
        return barrel, rod

    # boom cylinder: cab -> boom; stick cylinder: boom -> stick
    cylinder(cab, (1.3 * j(), 0.0, 1.2), boom, P0 + 0.45 * (P1 - P0) + np.array([0.0, 0.0, -0.25]), 60.0, 30.0)
    cylinder(boom, P0 + 0.7 * (P1 - P0) + np.array([0.0, 0.0, 0.45]), stick,
             P1 + np.array([-0.35, 0.0, 0.45]), 40.0, 20.0)
    # bucket linkage: link1 pinned to the stick, link2 pinned to the bucket,
    # joined at J; the bucket cylinder pushes on J
    L1 = P2 + 0.22 * (P1 - P2) + np.array([0.12, 0.0, 0.0])
    K = P2 + np.array([0.28, 0.0, -0.08])
    Jp = _circle_intersection(L1, 0.45 * j(), K, 0.42 * j(), side=1.0)
    link1 = _rod_body(B, L1, Jp, 0.5, width=0.06)
    link2 = _rod_body(B, Jp, K, 0.5, width=0.06)
    cylinder(stick, P1 + 0.3 * (P2 - P1) + np.array([0.25, 0.0, 0.1]), link1, Jp, 20.0, 10.0)
    B.joint(REVOLUTE, link1, stick, L1, ya)
    B.joint(REVOLUTE, link2, link1, Jp, ya)
    B.joint(REVOLUTE, link2, bucket, K, ya)
    return B.scene(dt, reset_body=-1)


def excavator_batch(n_worlds, seed=1003, dt=2e-3):
    rng = np.random.default_rng(seed)
    return concat([excavator_world(rng, dt) for _ in range(n_worlds)])


def heterogeneous_batch(n_worlds, seed=1003, dt=2e-3):
    """An equal mix of four-bars (with the sliding box), bipeds and
    excavators, interleaved world by world (four-bar, biped, excavator, ...)."""
    rng = np.random.default_rng(seed)
    n_f = (n_worlds + 2) // 3
    n_b = (n_worlds + 1) // 3
    n_e = n_worlds // 3
    fb = fourbar_batch(n_f, seed=int(rng.integers(1 << 30)), dt=dt)
    bp = biped_batch(n_b, seed=int(rng.integers(1 << 30)), dt=dt)
    ex = excavator_batch(n_e, seed=int(rng.integers(1 << 30)), dt=dt)
    parts = []
    for k in range(n_f):
        parts.append(fb._one(k))
        if k < n_b:
            parts.append(bp._one(k))
        if k < n_e:
            parts.append(ex._one(k))
    return concat(parts, dt=dt, reset_height=0.2)


BIN_HALF = (0.15, 0.15)  # 0.3 m x 0.3 m bin (walls 0.3 m high)


def box_bin_world(rng, n_boxes=20, dt=2e-3, half=BIN_HALF):
    """``n_boxes`` free boxes above a bin: sides U[0.02, 0.1] m, density
    U[100, 5000] kg/m^3 (mass ratio up to ~6e3), friction U[0.3, 1.0], random
    orientation, at rest.  Boxes are dropped one by one at a random (x, y)
    that keeps their axis-aligned bounds inside the walls, just above every
    earlier box whose bounds overlap in x-y (so nothing starts in contact).
    No joints; contacts come from box-in-bin generation each step."""
    B = _Builder()
    placed = []  # (lo, hi) bounds
    box = []
    for _ in range(n_boxes):
        side = rng.uniform(0.02, 0.1, 3)
        h = 0.5 * side
        rho = rng.uniform(100.0, 5000.0)
        m = rho * side.prod()
        q = random_quat(rng)
        R = quat_to_mat(q)
        ext = np.abs(R) @ h
        x = rng.uniform(-half[0] + ext[0] + 1e-3, half[0] - ext[0] - 1e-3)
        y = rng.uniform(-half[1] + ext[1] + 1e-3, half[1] - ext[1] - 1e-3)
        z = ext[2] + 0.005
        for lo, hi in placed:
            if lo[0] < x + ext[0] and x - ext[0] < hi[0] and lo[1] < y + ext[1] and y - ext[1] < hi[1]:
                z = max(z, hi[2] + ext[2] + 0.005)
        c = np.array([x, y, z])
        placed.append((c - ext, c + ext))
        B.body(m, box_inertia(m, *side), c, q)
        box.append(np.r_[h, rng.uniform(0.3, 1.0)])
    s = B.scene(dt)
    s.body_box = np.array(box)
    return s


def box_bin_batch(n_worlds, seed=1005, n_boxes=20, dt=2e-3):
    rng = np.random.default_rng(seed)
    return concat([box_bin_world(rng, n_boxes, dt) for _ in range(n_worlds)])


def box_bin_resting_world(rng, dt=2e-3, half=BIN_HALF):
    """Twelve boxes already in contact, for single-step tests: six on the
    floor in a 3 x 2 grid (two of them against the -x and +x walls, unrotated),
    each carrying a smaller box of the same yaw on its top face.  Every
    contact penetrates by a draw from U[0, 2 mm]; vertex-face decisions stay
    at least 4 mm from their thresholds; 56 contacts in all."""
    B = _Builder()
    box = []
    cells = [(-0.1, -0.06), (0.0, -0.06), (0.1, -0.06), (-0.1, 0.06), (0.0, 0.06), (0.1, 0.06)]
    for i, (cx, cy) in enumerate(cells):
        side = rng.uniform(0.04, 0.06, 3)
        h = 0.5 * side
        wall = i in (0, 2)
        yaw = 0.0 if wall else rng.uniform(0, 2 * np.pi)
        q = quat_axis_angle((0.0, 0.0, 1.0), yaw)
        d = rng.uniform(0.0, 0.002)
        if wall:
            sgn = -1.0 if i == 0 else 1.0
            cx = sgn * (half[0] - h[0] + rng.uniform(0.0, 0.002))
        c = np.array([cx, cy, h[2] - d])
        rho = rng.uniform(100.0, 5000.0)
        m = rho * side.prod()
        lo = B.body(m, box_inertia(m, *side), c, q)
        box.append(np.r_[h, rng.uniform(0.3, 1.0)])
        # the smaller box on top, same yaw, footprint 5-10 mm inside each side
        hu = np.r_[h[:2] - rng.uniform(0.005, 0.01, 2), rng.uniform(0.01, 0.03)]
        du = rng.uniform(0.0, 0.002)
        cu = np.array([c[0], c[1], c[2] + h[2] + hu[2] - du])
        mu_ = rng.uniform(100.0, 5000.0) * 8 * hu.prod()
        B.body(mu_, box_inertia(mu_, *(2 * hu)), cu, q)
        box.append(np.r_[hu, rng.uniform(0.3, 1.0)])
        _ = lo
    s = B.scene(dt)
    s.body_box = np.array(box)
    return s


def box_bin_resting_batch(n_worlds, seed=1005, dt=2e-3):
    rng = np.random.default_rng(seed)
    return concat([box_bin_resting_world(rng, dt) for _ in range(n_worlds)])


def perturb_state(scene, rng, v_scale=0.2, w_scale=0.5):
    """Random twists (not constraint-consistent) for single-step problems."""
    s = scene.replace(u=scene.u.copy())
    s.u[:, :3] += rng.normal(0.0, v_scale, (scene.n_bodies, 3))
    s.u[:, 3:] += rng.normal(0.0, w_scale, (scene.n_bodies, 3))
    return s


def round_to_f32(scene):
    """The same scene with every floating-point field rounded to FP32 and
    quaternions renormalised in FP32, so that FP32 and FP64 consumers see
    identical inputs."""
    f = {}
    for fld in dataclasses.fields(scene):
        v = getattr(scene, fld.name)
        if isinstance(v, np.ndarray) and v.dtype == np.float64:
            f[fld.name] = v.astype(np.float32).astype(np.float64)
    s = scene.replace(**f)
    return s


# ----------------------------------------------------------------------------
# counter-based random numbers: Philox4x32-10 (Salmon et al., SC'11)
# ----------------------------------------------------------------------------

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint32(0x9E3779B9)
PHILOX_W1 = np.uint32(0xBB67AE85)


def philox4x32(counter, key, rounds=10):
    """Philox4x32 with ``rounds`` rounds.  ``counter``: uint32 array [..., 4];
    ``key``: uint32 array [..., 2].  Returns uint32 [..., 4]."""
    c = np.asarray(counter, np.uint32).copy()
    k = np.asarray(key, np.uint32).copy()
    c0, c1, c2, c3 = (c[..., i].astype(np.uint64) for i in range(4))
    k0 = k[..., 0].astype(np.uint64)
    k1 = k[..., 1].astype(np.uint64)
    mask = np.uint64(0xFFFFFFFF)
    for r in range(rounds):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        n0 = (hi1 ^ c1 ^ k0) & mask
        n1 = lo1
        n2 = (hi0 ^ c3 ^ k1) & mask
        n3 = lo0
        c0, c1, c2, c3 = n0, n1, n2, n3
        if r + 1 < rounds:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_normal_pair(seed, world, step, slot):
    """Two standard normals from Philox4x32-10 at counter (world, step, slot, 0)
    with key (seed_lo, seed_hi), through the Box-Muller transform computed in
    FP32 (the uniform u1 is taken in (0, 1], u2 in [0, 1))."""
    world = np.asarray(world, np.uint32)
    step = np.asarray(step, np.uint32)
    slot = np.asarray(slot, np.uint32)
    shape = np.broadcast(world, step, slot).shape
    ctr = np.zeros(shape + (4,), np.uint32)
    ctr[..., 0] = world
    ctr[..., 1] = step
    ctr[..., 2] = slot
    key = np.zeros(shape + (2,), np.uint32)
    key[..., 0] = np.uint32(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint32((seed >> 32) & 0xFFFFFFFF)
    r = philox4x32(ctr, key)
    # 24-bit uniforms, exactly representable in FP32
    inv = np.float32(1.0 / 16777216.0)
    u1 = ((r[..., 0] >> np.uint32(8)).astype(np.float32) + np.float32(1.0)) * inv
    u2 = (r[..., 1] >> np.uint32(8)).astype(np.float32) * inv
    return u1, u2


# --- small worlds for tests --------------------------------------------------


def random_quat(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def random_chain_world(rng, n_bodies=4, with_limits=True, on_manifold=False, dt=1e-3):
    """Random bodies in random poses joined in a chain (first to the world)
    by revolute or prismatic joints whose frames are random, so the
    constraints are generally violated (off the manifold) unless
    ``on_manifold``; used for finite-difference checks."""
    B = _Builder()
    for i in range(n_bodies):
        m = rng.uniform(0.2, 3.0)
        B.body(m, rng.uniform(0.01, 0.2, 3) * m, rng.normal(0, 0.5, 3), random_quat(rng),
               rng.normal(0, 0.5, 3), rng.normal(0, 1.0, 3))
    for i in range(n_bodies):
        jt = int(rng.integers(0, 2))
        a, b = i, i - 1
        lim = (np.nan, np.nan)
        if with_limits and rng.uniform() < 0.6:
            lo = rng.uniform(-1.0, 0.0)
            hi = rng.uniform(0.0, 1.0)
            lim = (lo, hi) if rng.uniform() < 0.5 else ((lo, np.nan) if rng.uniform() < 0.5 else (np.nan, hi))
        if on_manifold:
            pw = rng.normal(0, 0.5, 3)
            B.joint(jt, a, b, pw, rng.normal(size=3), limit=lim)
        else:
            fa = np.concatenate([rng.normal(0, 0.2, 3), random_quat(rng)])
            fb = np.concatenate([rng.normal(0, 0.2, 3), random_quat(rng)])
            B.jt.append(jt)
            B.jb.append((a, b))
            B.jf.append(np.concatenate([fa, fb]))
            B.jl.append(np.asarray(lim, np.float64))
            B.ja.append(1)
    return B.scene(dt)


def box_point_contacts(rng, n_points=3, mu=0.0, dt=1e-3, gap_scale=0.0, v_scale=0.5):
    """A free box above z = 0 touching the ground at ``n_points`` random
    points of its lower face (optionally with small random gaps), moving with
    a random twist: a small contact problem with a unique solution when the
    points are not collinear."""
    B = _Builder()
    sx, sy, sz = rng.uniform(0.1, 0.3, 3)
    m = rng.uniform(0.5, 2.0)
    q = quat_axis_angle(rng.normal(size=3), rng.uniform(0, 0.05))
    R = quat_to_mat(q)
    pts_local = np.stack([rng.uniform(-0.5, 0.5, n_points) * sx, rng.uniform(-0.5, 0.5, n_points) * sy,
                          np.full(n_points, -0.5 * sz)], axis=1)
    lowest = min((R @ p)[2] for p in pts_local)
    com = np.array([0.0, 0.0, -lowest])
    box = B.body(m, box_inertia(m, sx, sy, sz), com, q, rng.normal(0, v_scale, 3), rng.normal(0, v_scale, 3))
    for k, pl in enumerate(pts_local):
        pw = com + R @ pl
        gap = max(pw[2], 0.0) + rng.uniform(0.0, gap_scale)
        B.contact(box, -1, (pw[0], pw[1], pw[2]), (0.0, 0.0, 1.0), gap, mu, k)
    return B.scene(dt)
