"""Pins of the oracle parts that the closed forms of the other oracle tests
do not reach:

* the restart rule of the accelerated iteration (Alg. 1 step 8; Sec. 4.1
  Nesterov acceleration with restart, after Goldstein, O'Donoghue, Setzer
  and Baraniuk 2014): two decoupled unit-diagonal rows reduce Alg. 1 to two
  scalar recurrences, worked out by hand below;
* the pose update of the semi-implicit Euler step (Sec. 3, exponential map
  on SO(3)): a rotation about a world axis in closed form, angular momentum
  of a torque-free body, energy drift and the small-angle period of a
  pendulum, each converging with the time step;
* joint actuation (a generalized force along the joint coordinate) on a
  hinge and a slider, in closed form;
* an active joint limit (Sec. 3 unilateral limits): a pendulum held on its
  stop;
* where the impulses are not unique and where the dual residual has a floor
  (redundant loop rows, Sec. 3 and Sec. 4): the rank and floor report.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from paper_2603_16536_amd import scenes

TIGHT = dict(eps=1e-13, max_iters=200000)


def rot(q):
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


# ---------------------------------------------------------------------------
# restart rule
# ---------------------------------------------------------------------------


def two_row_reduction(n_iters, eta, rho_a, rho_b, gamma):
    """Alg. 1 on D~ = I with row a free (v~_a = -1) and row b a limit row
    that separates (v~_b = +1/2), cold start, worked out by hand.

    Row a (free): the projection is the identity, so y = x - z^/rho and
    z = z^ - rho (x - y) = 0 at every iteration; hence z^ = 0 and y = x, and
    step 5 reads x_k = (1 + eta x_{k-1} + rho_a y^_{k-1}) / (1 + eta + rho_a).
    Row b (limit): while x_k - z^_{k-1}/rho_b <= 0 the projection gives
    y = 0 (so y^ = 0) and step 5 reads x_k = (-1/2 + eta x_{k-1} +
    z^_{k-1}) / (1 + eta + rho_b), step 7 z_k = z^_{k-1} - rho_b x_k.
    Step 8: c_k = rho_a (y_k - y^_{k-1})^2 + (z_k - z^_{k-1})^2 / rho_b (the
    other two terms vanish).  No restart when c_k < gamma c_prev:
    a+ = (1 + sqrt(1 + 4 a^2)) / 2, beta = (a - 1) / a+, y^_k = y_k + beta
    (y_k - y_{k-1}) and z^ likewise, c_prev = c_k.  Restart otherwise:
    a = 1, y^_k = y_{k-1}, z^_k = z_{k-1}, c_prev = c_prev / gamma.
    Returns per iteration (restart, x_a, x_b, z_b)."""
    xa = yha = ypa = 0.0
    xb = zhb = zpb = 0.0
    a, c_prev = 1.0, math.inf
    out = []
    for _ in range(n_iters):
        xa_n = (1.0 + eta * xa + rho_a * yha) / (1.0 + eta + rho_a)
        xb_n = (-0.5 + eta * xb + zhb) / (1.0 + eta + rho_b)
        assert xb_n - zhb / rho_b <= 0.0  # the reduction's premise: y_b stays 0
        zb_n = zhb - rho_b * xb_n
        c = rho_a * (xa_n - yha) ** 2 + (zb_n - zhb) ** 2 / rho_b
        restart = not c < gamma * c_prev
        if not restart:
            a_n = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a * a))
            beta = (a - 1.0) / a_n
            yha = xa_n + beta * (xa_n - ypa)
            zhb = zb_n + beta * (zb_n - zpb)
            a, c_prev = a_n, c
        else:
            yha, zhb = ypa, zpb
            a, c_prev = 1.0, c_prev / gamma
        xa, ypa, xb, zpb = xa_n, xa_n, xb_n, zb_n
        out.append((int(restart), xa_n, xb_n, zb_n))
    return out


# Parameter set A has the default restart factor and penalties that differ
# per row (so the rho and 1/rho weights of c matter); set B has a restart
# factor of 0.9, where the c_prev / gamma of a restart changes which later
# iterations restart.  Hand-worked outcome over the first 25 iterations (c
# stays far above rounding there): set A restarts at 5, 10, 15, 20 and 25,
# set B at 8, 9, 10, 18, 19 and 20.
SETS = {"A": (0.1, 0.5, 1.0, 0.999), "B": (0.1, 0.5, 0.3, 0.9)}


@pytest.mark.parametrize("name", sorted(SETS))
def test_restart_rule_on_two_decoupled_rows(orc, name):
    eta, ra, rb, gamma = SETS[name]
    # physical problem whose Jacobi scaling gives D~ = I, v~ = (-1, 1/2)
    D = np.diag([4.0, 0.25])
    vf = np.array([-2.0, 0.25])  # p = (1/2, 2)
    kind = np.array([orc.ROW_BILATERAL, orc.ROW_LIMIT], np.int32)
    mu = np.zeros(2)
    ref = two_row_reduction(25, eta, ra, rb, gamma)
    assert [k + 1 for k, r in enumerate(ref) if r[0]] == {"A": [5, 10, 15, 20, 25], "B": [8, 9, 10, 18, 19, 20]}[name]
    P = orc.Params(eta=eta, rho_bil=ra, rho_c=rb, restart_factor=gamma, eps=0.0)
    for k in (1, 2, 4, 5, 6, 8, 9, 10, 11, 15, 19, 20, 21, 24, 25):
        o = orc.solve_ncp(D, vf, kind, mu, P.replace(fixed_iters=k), log_iters=k)
        rs, xa, xb, zb = ref[k - 1]
        assert list(o["restart_log"]) == [r[0] for r in ref[:k]], k
        # y_a = x_a, y_b = 0; r_p = |x_b|; r_d = max(|x_a - 1|, |x_b + 1/2 - z_b|)
        assert abs(o["lam_tilde"][0] - xa) < 1e-13
        assert o["lam_tilde"][1] == 0.0
        assert abs(o["lam"][0] - 0.5 * xa) < 1e-13
        assert abs(o["resid"][0] - abs(xb)) < 1e-13
        assert abs(o["resid"][1] - max(abs(xa - 1.0), abs(xb + 0.5 - zb))) < 1e-13


# ---------------------------------------------------------------------------
# pose update
# ---------------------------------------------------------------------------


def free_body(dt, inertia, q0, v, w, mass=2.0, pos=(0.0, 0.0, 1.0)):
    B = scenes._Builder()
    B.body(mass, inertia, pos, q0, v=v, w=w)
    return B.scene(dt, gravity=(0.0, 0.0, 0.0))


@pytest.mark.parametrize("w", [(0.0, 0.0, 3.0), (1.5, -2.0, 0.7)])
def test_single_step_pose_is_world_frame_exponential_map(orc, w):
    """Isotropic inertia, no gravity: the twist is unchanged and the pose
    advances by r+ = r + dt v and R+ = exp(dt [w]x) R (world-frame angular
    velocity, left multiplication)."""
    dt = 1e-2
    q0 = scenes.quat_axis_angle((1.0, 0.0, 0.0), 0.5 * math.pi)
    s = free_body(dt, (0.3, 0.3, 0.3), q0, v=(0.2, -0.1, 0.4), w=w)
    out = orc.step(s, orc.Params(dt=dt, gravity=(0.0, 0.0, 0.0)))
    assert np.abs(out["u"] - s.u).max() < 1e-15
    assert np.abs(out["q"][0, :3] - (s.q[0, :3] + dt * s.u[0, :3])).max() < 1e-15
    R_exp = expm(dt * skew(np.asarray(w))) @ rot(q0)
    assert np.abs(rot(out["q"][0, 3:]) - R_exp).max() < 1e-14
    assert abs(np.linalg.norm(out["q"][0, 3:]) - 1.0) < 1e-15


def rollout(orc, s, P, n, observe):
    q, u = s.q.copy(), s.u.copy()
    vals = [observe(q, u)]
    for _ in range(n):
        o = orc.step(s, P, q=q, u=u)
        q, u = o["q"], o["u"]
        vals.append(observe(q, u))
    return vals


def test_torque_free_body_conserves_angular_momentum_to_first_order(orc):
    """A torque-free body with three different principal moments tumbles
    with constant world angular momentum R I R^T w; the explicit gyroscopic
    term and the exponential map keep it to O(dt) over a fixed time."""
    q0 = scenes.quat_axis_angle((1.0, 0.0, 0.0), 0.7)
    inertia = (0.1, 0.2, 0.35)
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        s = free_body(dt, inertia, q0, v=(0.1, 0.0, 0.0), w=(3.0, 1.0, -2.0))
        P = orc.Params(dt=dt, gravity=(0.0, 0.0, 0.0))

        def L(q, u):
            R = rot(q[0, 3:])
            return R @ np.diag(inertia) @ R.T @ u[0, 3:]

        Ls = np.array(rollout(orc, s, P, int(round(0.5 / dt)), L))
        errs.append(np.abs(Ls - Ls[0]).max() / np.linalg.norm(Ls[0]))
    assert errs[1] < 3e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert 1.8 < e0 / e1 < 2.2


def pendulum_energy(s, q, u):
    m = s.body_mass[0]
    R = rot(q[0, 3:])
    I = R @ np.diag(s.body_inertia[0]) @ R.T
    return 0.5 * m * u[0, :3] @ u[0, :3] + 0.5 * u[0, 3:] @ I @ u[0, 3:] + m * 9.81 * q[0, 2]


def test_pendulum_energy_drift_is_first_order(orc):
    """Invariant: without contact and without stabilisation, the energy
    error of the hinged rod over one second falls in proportion to dt."""
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        s = scenes.pendulum(length=0.5, mass=1.3, theta0=1.0, dt=dt)
        P = orc.Params(dt=dt, baumgarte=0.0, **TIGHT)
        E = np.array(rollout(orc, s, P, int(round(1.0 / dt)), lambda q, u: pendulum_energy(s, q, u)))
        errs.append(np.abs(E - E[0]).max() / abs(E[0]))
    assert errs[1] < 2e-2
    for e0, e1 in zip(errs, errs[1:]):
        assert 1.8 < e0 / e1 < 2.2


def test_pendulum_small_angle_period(orc):
    """Period of the hinged rod at 0.02 rad amplitude against the textbook
    2 pi sqrt(I_p / (m g d)) (with the finite-amplitude factor 1 + th^2/16):
    the error falls at least in proportion to dt."""
    L, m, g, th0 = 0.5, 1.3, 9.81, 0.02
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        s = scenes.pendulum(length=L, mass=m, theta0=th0, dt=dt)
        P = orc.Params(dt=dt, baumgarte=0.0, **TIGHT)
        th = np.array(rollout(orc, s, P, int(round(4.0 / dt)), lambda q, u: math.atan2(q[0, 0], -q[0, 2])))
        t = np.arange(len(th)) * dt
        up = [t[k] + dt * (-th[k]) / (th[k + 1] - th[k]) for k in range(len(th) - 1) if th[k] < 0.0 <= th[k + 1]]
        assert len(up) >= 3
        period = np.diff(up).mean()
        Ip = s.body_inertia[0, 1] + m * (0.5 * L) ** 2  # rod inertia about the hinge (world y)
        T = 2 * math.pi * math.sqrt(Ip / (m * g * 0.5 * L)) * (1.0 + th0 * th0 / 16.0)
        errs.append(abs(period - T) / T)
    assert errs[0] < 1e-5
    for e0, e1 in zip(errs, errs[1:]):
        assert e0 / e1 > 1.9


# ---------------------------------------------------------------------------
# actuation and limits
# ---------------------------------------------------------------------------


def hinged_rod(theta0, omega0=0.0, limit=(np.nan, np.nan), dt=1e-3, L=0.5, m=1.3):
    """scenes.pendulum with an optional limit on the hinge coordinate (0 in
    the pose built here)."""
    B = scenes._Builder()
    d = np.array([math.sin(theta0), 0.0, -math.cos(theta0)])
    wv = np.array([0.0, -omega0, 0.0])
    rod = scenes._rod_body(B, np.zeros(3), L * d, m, 0.02, v=np.cross(wv, 0.5 * L * d), w=wv)
    B.joint(scenes.REVOLUTE, rod, -1, np.zeros(3), (0.0, 1.0, 0.0), limit=limit)
    return B.scene(dt)


@pytest.mark.parametrize("gravity", [0.0, 9.81])
@pytest.mark.parametrize("tau", [0.7, -1.9])
def test_hinge_torque_closed_form(orc, tau, gravity):
    """A generalized force tau on the hinge (axis x of the joint frames =
    world +y) turns the rod about +y: I_p w+ = I_p w- + dt (tau + moment
    of gravity about the pivot), v+ = w+ x c; the joint coordinate grows
    with positive rotation of the rod about the axis."""
    dt, L, m = 1e-3, 0.5, 1.3
    s = hinged_rod(1.1, omega0=-0.8, dt=dt, L=L, m=m)
    P = orc.Params(dt=dt, gravity=(0.0, 0.0, -gravity), baumgarte=0.0, **TIGHT)
    out = orc.step(s, P, joint_torque=np.array([tau]))
    e = np.array([0.0, 1.0, 0.0])
    c = s.q[0, :3]
    Ip = s.body_inertia[0, 1] + m * (c @ c)
    moment = e @ np.cross(c, np.array([0.0, 0.0, -gravity * m]))
    w_plus = s.u[0, 3:] @ e + dt * (tau + moment) / Ip
    assert np.abs(out["u"][0, 3:] - w_plus * e).max() < 1e-10
    assert np.abs(out["u"][0, :3] - w_plus * np.cross(e, c)).max() < 1e-10
    c0 = orc.joint_coordinate(s, s.q, 0)[0]
    c1 = orc.joint_coordinate(s, out["q"], 0)[0]
    assert abs((c1 - c0) - dt * w_plus) < 1e-9


@pytest.mark.parametrize("force", [3.0, -0.4])
def test_slider_force_closed_form(orc, force):
    """A prismatic joint to the world along world x: the generalized force F
    accelerates the slider by F / m along the axis, gravity is carried by
    the joint, and the coordinate (offset along the axis) grows with it."""
    dt, m = 1e-3, 0.8
    B = scenes._Builder()
    body = B.body(m, (0.01, 0.02, 0.03), (0.0, 0.0, 0.5), (0.0, 0.0, 0.0, 1.0), v=(0.3, 0.0, 0.0))
    B.joint(scenes.PRISMATIC, body, -1, (0.0, 0.0, 0.5), (1.0, 0.0, 0.0))
    s = B.scene(dt)
    out = orc.step(s, orc.Params(dt=dt, baumgarte=0.0, **TIGHT), joint_torque=np.array([force]))
    v_plus = 0.3 + dt * force / m
    assert np.abs(out["u"][0] - np.array([v_plus, 0, 0, 0, 0, 0])).max() < 1e-10
    assert abs(orc.joint_coordinate(s, out["q"], 0)[0] - orc.joint_coordinate(s, s.q, 0)[0] - dt * v_plus) < 1e-10


def test_pendulum_held_on_its_stop(orc):
    """The rod horizontal (theta = 90 degrees) at rest, gravity turning it
    about +y, i.e. toward larger joint coordinates.  An upper bound at the
    current coordinate stops it: w+ = 0, v+ = 0, and the limit row carries
    the whole moment of gravity about the pivot, dt m g L/2 (N m s).  A lower
    bound at the same coordinate does not act: the rod swings as if free."""
    dt, L, m, g = 1e-3, 0.5, 1.3, 9.81
    P = orc.Params(dt=dt, baumgarte=0.2, eta=1e-9, rho_bil=1e-9, rho_c=1.0, **TIGHT)
    held = hinged_rod(0.5 * math.pi, limit=(np.nan, 0.0), dt=dt, L=L, m=m)
    out = orc.step(held, P)
    assert out["status"][0] == orc.OK
    assert np.abs(out["u"]).max() < 1e-10
    S = orc.world_system(held, P, 0)
    assert S["kind"][5] == orc.ROW_LIMIT and S["J"].shape[0] == 6
    assert abs(out["lam"][5] - dt * m * g * 0.5 * L) < 1e-10
    free = hinged_rod(0.5 * math.pi, limit=(0.0, np.nan), dt=dt, L=L, m=m)
    out_free = orc.step(free, P)
    out_none = orc.step(hinged_rod(0.5 * math.pi, dt=dt, L=L, m=m), P)
    assert abs(out_free["lam"][5]) < 1e-12
    assert np.abs(out_free["u"] - out_none["u"]).max() < 1e-10
    Ip = held.body_inertia[0, 1] + m * (0.5 * L) ** 2
    assert abs(out_free["u"][0, 4] - dt * m * g * 0.5 * L / Ip) < 1e-10


# ---------------------------------------------------------------------------
# rank and floor report
# ---------------------------------------------------------------------------


def test_rank_report_matches_mobility(orc):
    """Maximal-coordinate mobility 6 n_b - rank(J) equals the mechanism's
    degrees of freedom: 1 for the four-bar (3 moving links: rank 17 of its
    20 bilateral rows, 3 redundant planar-loop rows) and 16 for the biped
    (6 for the floating pelvis + 10 chain joints: rank 170 of 200)."""
    P = orc.Params(dt=1e-3)
    fb = scenes.fourbar_batch(1, seed=1001, with_box=False)
    r = orc.floor_report(fb, P, 0)
    assert (r["m"], r["rank_JB"], r["rank_J"], r["null_dim"]) == (20, 17, 17, 3)
    bp = scenes.biped_batch(1)
    bp = bp.replace(contact_world=np.zeros(0, np.int32), contact_body=np.zeros((0, 2), np.int32),
                    contact_point=np.zeros((0, 3)), contact_normal=np.zeros((0, 3)), contact_gap=np.zeros(0),
                    contact_mu=np.zeros(0), contact_key=np.zeros(0, np.int32))
    r = orc.floor_report(bp, P.replace(dt=2e-3), 0)
    assert r["m"] == 200 and r["rank_JB"] == 170 and 6 * 31 - r["rank_JB"] == 16
    # assembled exactly: the bias is consistent, no floor
    assert r["floor_inf"] < 1e-9


def test_floor_of_a_duplicated_row_is_reached_by_padmm(orc):
    """Two copies of one bilateral row with different biases a, b (after
    scaling): no impulse can satisfy both, null(D~) = span(1, -1), and the
    smallest reachable infinity norm of the constraint velocity is |a - b|/2.
    The report gives exactly that, and Alg. 1 stalls there."""
    j = np.array([0.3, -1.2, 0.5])
    Minv = np.diag([2.0, 0.5, 1.0])
    d = j @ Minv @ j
    D = np.array([[d, d, 0.0], [d, d, 0.0], [0.0, 0.0, 1.0]])
    a, b = 0.8, -0.3
    vf = np.array([a, b, 0.4]) * math.sqrt(d) * np.array([1.0, 1.0, 1.0 / math.sqrt(d)])
    kind = np.array([orc.ROW_BILATERAL] * 3, np.int32)
    out = orc.solve_ncp(D, vf, kind, np.zeros(3), orc.Params(eta=1e-3, rho_bil=1e-3, eps=1e-14, max_iters=20000))
    assert out["status"] == orc.MAXITER
    assert abs(out["resid"][1] - abs(a - b) / 2) < 1e-9
    # the same floor from the report's formula on this D~, v~
    p = 1.0 / np.sqrt(np.diag(D))
    ev, V = np.linalg.eigh(p[:, None] * D * p[None, :])
    N = V[:, ev < 1e-9]
    n = N @ (N.T @ (p * vf))
    assert abs(n @ n / np.abs(n).sum() - abs(a - b) / 2) < 1e-12


def test_rounded_loop_frames_set_the_excavator_floor(orc):
    """The excavator's rounded joint frames (FP32 inputs) leave a bias
    component outside range(D~_BB): the reported floor is above 1e-6, at
    most the dual residual the oracle stalls at, and the FP64-assembled
    excavator (12 redundant rows: three per planar loop) has none."""
    ex = scenes.excavator_batch(2, seed=1003)
    P = orc.Params(dt=2e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-6, max_iters=2000, baumgarte=0.2)
    rex = scenes.round_to_f32(ex)
    out = orc.step(rex, P)
    for w in range(2):
        exact = orc.floor_report(ex, P, w)
        rounded = orc.floor_report(rex, P, w)
        assert exact["floor_inf"] < 1e-9
        assert rounded["floor_inf"] > 1e-6
        assert rounded["floor_inf"] <= out["resid"][w, 1] * (1 + 1e-9)
        # four planar loops, three redundant rows each
        assert exact["null_dim"] == 12
