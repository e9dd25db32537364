"""Pins of the oracle's joint drives and of its Moreau-Jean midpoint variant.

Drives (Sec. 3: implicit PD with the gains absorbed into the constraint
rows, armature and viscous damping handled likewise; Eq. 2: their R and v*
terms).  A driven joint gets one row along its coordinate; one step of a
hinge or a slider whose only free degree of freedom is that coordinate has
the closed form of backward-Euler PD on a single inertia:

    (I + I_a + hz dt kp + dt (kd + d)) cdot+ = (I + I_a) cdot- + dt tau
                                               + dt kp (ref - c)

with I the body's inertia about the axis (mass for a slider), I_a the
armature, d the damping, tau any explicit generalized force and hz the time
from the configuration c to the end of the step (dt, or dt / 2 from the
half-step configuration of the midpoint scheme).

Midpoint (Sec. 3, Moreau-Jean): forces and constraints at q + dt/2 u-, then
u+, then q+ = q_mid + dt/2 u+.  A body in free flight under gravity then
follows the exact parabola, while semi-implicit Euler is off by t dt g / 2.
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


def hinge_wheel(drive, omega0, dt, angle0=0.0):
    """A wheel (3-axis inertia) on a hinge to the world about world y
    through its centre: the hinge coordinate is its only degree of freedom
    and gravity exerts no moment about the axis."""
    B = scenes._Builder()
    q0 = scenes.quat_axis_angle((0.0, 1.0, 0.0), angle0)
    wheel = B.body(2.0, (0.03, 0.05, 0.04), (0.0, 0.0, 0.5), (0.0, 0.0, 0.0, 1.0))
    B.joint(scenes.REVOLUTE, wheel, -1, (0.0, 0.0, 0.5), (0.0, 1.0, 0.0), drive=drive)
    s = B.scene(dt)
    # rotate the wheel after assembly, so the coordinate starts at angle0
    s.q[0, 3:] = q0
    s.u[0] = (0.0, 0.0, 0.0, 0.0, omega0, 0.0)
    return s


@pytest.mark.parametrize("kp,kd,damp,arm,ref,tau", [
    (15.0, 0.6, 0.0, 0.0, 0.4, 0.0),      # the paper's RL gains
    (15.0, 0.6, 0.2, 0.01, -0.3, 0.5),    # with damping, armature and an explicit torque
    (0.0, 0.0, 0.0, 0.02, 0.0, 1.7),      # armature alone
    (2e4, 5.0, 0.0, 0.0, 0.1, 0.0),       # stiff
])
def test_hinge_drive_closed_form(orc, kp, kd, damp, arm, ref, tau):
    dt, w0, c0 = 2e-3, 1.3, 0.25
    s = hinge_wheel((kp, kd, damp, arm, ref), w0, dt, angle0=c0)
    c = orc.joint_coordinate(s, s.q, 0)[0]
    assert abs(c - c0) < 1e-12  # positive rotation about the axis raises the coordinate
    P = orc.Params(dt=dt, baumgarte=0.0, eta=1e-10, rho_bil=1e-10, **TIGHT)
    out = orc.step(s, P, joint_torque=np.array([tau]))
    assert out["status"][0] == orc.OK
    I = s.body_inertia[0, 1]
    w_plus = ((I + arm) * w0 + dt * tau + dt * kp * (ref - c)) / (I + arm + dt * dt * kp + dt * (kd + damp))
    assert abs(out["u"][0, 4] - w_plus) < 1e-10 * max(1.0, abs(w_plus))
    assert np.abs(out["u"][0, [0, 1, 2, 3, 5]]).max() < 1e-10
    # the drive row is the sixth row; its impulse is what turned the wheel
    assert abs(out["lam"][5] - (I * (w_plus - w0) - dt * tau)) < 1e-9 * max(1.0, abs(out["lam"][5]))
    S = orc.world_system(s, P, 0)
    assert S["R"][5] > 0.0 and np.all(S["R"][:5] == 0.0)


def test_stiff_implicit_drive_stays_stable_where_explicit_pd_diverges(orc):
    """kp = 2e5 N m/rad on a 0.05 kg m^2 wheel at dt = 2 ms: omega dt = 4,
    past the stability bound 2 of an explicit spring under the symplectic
    (semi-implicit) Euler step; as a drive row the wheel settles on the
    reference, as an explicit generalized force its rate grows without
    bound."""
    dt, kp, ref = 2e-3, 2e5, 0.2
    P = orc.Params(dt=dt, baumgarte=0.0, eta=1e-10, rho_bil=1e-10, **TIGHT)
    s = hinge_wheel((kp, 0.0, 0.0, 0.0, ref), 0.0, dt)
    assert math.sqrt(kp / s.body_inertia[0, 1]) * dt == pytest.approx(4.0)
    q, u = s.q.copy(), s.u.copy()
    errs = []
    for _ in range(100):
        o = orc.step(s, P, q=q, u=u)
        q, u = o["q"], o["u"]
        errs.append(orc.joint_coordinate(s, q, 0)[0] - ref)
    errs = np.array(errs)
    # decays from the initial error ref (backward Euler damps the spring)
    assert abs(errs[-1]) < 1e-6 and np.abs(errs).max() < ref
    s0 = hinge_wheel((0.0, 0.0, 0.0, 0.0, 0.0), 0.0, dt)
    q, u = s0.q.copy(), s0.u.copy()
    rates = []
    for _ in range(20):
        c, Ja, _ = orc.joint_coordinate(s0, q, 0)
        o = orc.step(s0, P, q=q, u=u, joint_torque=np.array([kp * (ref - c)]))
        q, u = o["q"], o["u"]
        rates.append(abs(u[0, 4]))
    assert rates[-1] > 5 * rates[0] and rates[-1] > 1e4


def test_free_flight_midpoint_is_exact_and_euler_lags(orc):
    """A torque-free body with isotropic inertia under gravity: after n
    steps the midpoint variant sits on r0 + t v0 + t^2 g / 2 and
    R = exp(t [w]x) R0 to rounding; semi-implicit Euler sits t dt g / 2
    further along g (sum of dt v_k with v_k = v0 + k dt g)."""
    dt, n = 1e-2, 50
    g = np.array([0.0, 0.0, -9.81])
    B = scenes._Builder()
    q0 = scenes.quat_axis_angle((0.3, 0.4, 0.5), 0.9)
    B.body(1.5, (0.2, 0.2, 0.2), (0.1, -0.2, 2.0), q0, v=(0.7, 0.1, 3.0), w=(0.4, -1.1, 2.0))
    s = B.scene(dt, gravity=tuple(g))
    t = n * dt
    r_exact = s.q[0, :3] + t * s.u[0, :3] + 0.5 * t * t * g
    R_exact = expm(t * skew(s.u[0, 3:])) @ rot(q0)
    for integ, r_expect in ((1, r_exact), (0, r_exact + 0.5 * t * dt * g)):
        P = orc.Params(dt=dt, gravity=tuple(g), integrator=integ)
        q, u = s.q.copy(), s.u.copy()
        for _ in range(n):
            o = orc.step(s, P, q=q, u=u)
            q, u = o["q"], o["u"]
        assert np.abs(q[0, :3] - r_expect).max() < 1e-12, integ
        assert np.abs(rot(q[0, 3:]) - R_exact).max() < 1e-12, integ
        assert np.abs(u[0, :3] - (s.u[0, :3] + t * g)).max() < 1e-12


def test_midpoint_configuration_and_rows(orc):
    """The midpoint variant evaluates the rows at q + dt/2 u-: positions
    advanced by dt/2 v, orientations by exp(dt/2 [w]x), and the Jacobian and
    Baumgarte bias over the remaining dt/2 are those of that configuration."""
    dt = 1e-2
    s = scenes.pendulum(length=0.5, mass=1.3, theta0=0.8, omega0=2.0, dt=dt)
    qm = orc.step_configuration(s, orc.Params(dt=dt, integrator=1))
    assert np.abs(qm[0, :3] - (s.q[0, :3] + 0.5 * dt * s.u[0, :3])).max() < 1e-15
    assert np.abs(rot(qm[0, 3:]) - expm(0.5 * dt * skew(s.u[0, 3:])) @ rot(s.q[0, 3:])).max() < 1e-14
    mid = orc.world_system(s, orc.Params(dt=dt, integrator=1, baumgarte=0.2), 0)
    at_qm = orc.world_system(s.replace(q=qm), orc.Params(dt=dt, baumgarte=0.2), 0)
    assert np.abs(mid["J"] - at_qm["J"]).max() < 1e-15
    # the anchor drifted off the pivot along the tangent: f != 0, bias over dt/2
    assert np.abs(at_qm["f"]).max() > 1e-6
    assert np.abs(mid["vstar"] - 2.0 * at_qm["vstar"]).max() < 1e-12


def test_midpoint_slider_spring_closed_form(orc):
    """A slider on a prismatic joint along world x with an implicit spring
    (kp, kd) toward ref: c_mid = c + dt/2 cdot-, then
    (m + dt/2 dt kp + dt kd) cdot+ = m cdot- + dt kp (ref - c_mid), and
    c+ = c_mid + dt/2 cdot+."""
    dt, m, kp, kd, ref, v0 = 5e-3, 0.8, 300.0, 2.0, 0.05, 0.4
    B = scenes._Builder()
    body = B.body(m, (0.01, 0.02, 0.03), (0.0, 0.0, 0.5), (0.0, 0.0, 0.0, 1.0), v=(v0, 0.0, 0.0))
    B.joint(scenes.PRISMATIC, body, -1, (0.0, 0.0, 0.5), (1.0, 0.0, 0.0), drive=(kp, kd, 0.0, 0.0, ref))
    s = B.scene(dt)
    P = orc.Params(dt=dt, baumgarte=0.0, eta=1e-10, rho_bil=1e-10, integrator=1, **TIGHT)
    out = orc.step(s, P)
    c_mid = 0.5 * dt * v0
    v_plus = (m * v0 + dt * kp * (ref - c_mid)) / (m + 0.5 * dt * dt * kp + dt * kd)
    assert abs(out["u"][0, 0] - v_plus) < 1e-10
    assert abs(orc.joint_coordinate(s, out["q"], 0)[0] - (c_mid + 0.5 * dt * v_plus)) < 1e-12
