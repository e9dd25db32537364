"""Pins of the oracle's time step against things the paper and mechanics
fix independently of its code:

* closed forms: one step of a hinged rod; the four-bar velocity update as an
  M-orthogonal projection onto the analytic one-DoF velocity space; a box on
  an incline that sticks for mu > tan(theta) and slides with the Coulomb
  deceleration for mu < tan(theta) (Sec. 3 contact law, Sec. 4 De Saxce
  claim that sliding leaves no normal velocity);
* the KKT system of Eq. 2 solved densely (bilateral problems);
* the minimum-norm limit of cold-started PADMM on redundant loops;
* exhaustive enumeration: 2^k active sets for frictionless contact, and
  separating / sticking / sliding modes for one frictional contact;
* the NCP conditions of Eq. 3 at the returned impulses;
* solver mechanics: warm-start fixed point, restart replay, status flags.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2603_16536_amd import scenes

TIGHT = dict(eps=1e-13, max_iters=200000)


def rot(q):
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def mass_matrix(scene):
    """Eq. 1, assembled here from the scene (not from the oracle)."""
    nb = scene.n_bodies
    M = np.zeros((6 * nb, 6 * nb))
    for i in range(nb):
        R = rot(scene.q[i, 3:])
        M[6 * i:6 * i + 3, 6 * i:6 * i + 3] = scene.body_mass[i] * np.eye(3)
        M[6 * i + 3:6 * i + 6, 6 * i + 3:6 * i + 6] = R @ np.diag(scene.body_inertia[i]) @ R.T
    return M


def forces(scene, g):
    """Newton-Euler h: gravity and the gyroscopic moment -w x (I w)."""
    M = mass_matrix(scene)
    h = np.zeros(6 * scene.n_bodies)
    for i in range(scene.n_bodies):
        w = scene.u[i, 3:]
        I = M[6 * i + 3:6 * i + 6, 6 * i + 3:6 * i + 6]
        h[6 * i:6 * i + 3] = scene.body_mass[i] * np.asarray(g)
        h[6 * i + 3:6 * i + 6] = -np.cross(w, I @ w)
    return M, h


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("theta0,omega0", [(0.3, 0.0), (1.1, -2.0), (-0.7, 1.5), (2.5, 0.4)])
def test_pendulum_single_step_closed_form(orc, theta0, omega0):
    L, m, dt, g0 = 0.5, 1.3, 1e-3, 9.81
    s = scenes.pendulum(length=L, mass=m, theta0=theta0, omega0=omega0, dt=dt)
    P = orc.Params(dt=dt, baumgarte=0.0, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    e = np.array([0.0, 1.0, 0.0])
    c = s.q[0, :3]  # COM relative to the pivot at the origin
    Ic = rot(s.q[0, 3:]) @ np.diag(s.body_inertia[0]) @ rot(s.q[0, 3:]).T
    Ip = e @ Ic @ e + m * np.dot(np.cross(e, c), np.cross(e, c))
    gvec = np.array([0.0, 0.0, -g0])
    w_minus = s.u[0, 3:] @ e
    w_plus = w_minus + dt * m * (e @ np.cross(c, gvec)) / Ip
    v_plus = w_plus * np.cross(e, c)
    assert np.abs(out["u"][0, 3:] - w_plus * e).max() < 1e-10
    assert np.abs(out["u"][0, :3] - v_plus).max() < 1e-10
    # textbook form about the pivot: I_p w+ = I_p w- - dt m g d sin(theta),
    # with w measured in the direction that increases theta (about -y)
    d = 0.5 * L
    assert abs(Ip * (-w_plus) - (Ip * (-w_minus) - dt * m * g0 * d * math.sin(theta0))) < 1e-10
    # net constraint impulse on the rod = momentum change minus gravity impulse
    J = orc.world_system(s, P, 0)["J"]
    imp = J.T @ out["lam"]
    assert np.abs(imp[:3] - (m * (v_plus - s.u[0, :3]) - dt * m * gvec)).max() < 1e-10


def fourbar_velocity_basis(scene):
    """Analytic one-DoF velocity basis T (18 x 1) of a planar four-bar
    (links: crank A-P, coupler P-Q, rocker D-Q; hinge axis e = world y) from
    the loop-closure velocity equations, with the crank rate set to 1."""
    g = scene.meta
    O = np.array([0.0, 0.0, 0.6])

    def w3(p2):
        return O + np.array([p2[0], 0.0, p2[1]])

    A, P, Q, D = w3(np.zeros(2)), w3(g["P"]), w3(g["Q"]), w3(g["D"])
    e = np.array([0.0, 1.0, 0.0])
    vP = np.cross(e, P - A)
    # vP + w3 e x (Q - P) = w4 e x (Q - D)   (x and z components)
    a1, a2 = np.cross(e, Q - P), np.cross(e, Q - D)
    Msys = np.array([[a1[0], -a2[0]], [a1[2], -a2[2]]])
    w3r, w4r = np.linalg.solve(Msys, -np.array([vP[0], vP[2]]))
    c1, c2, c3 = scene.q[0, :3], scene.q[1, :3], scene.q[2, :3]
    T = np.zeros(18)
    T[0:3], T[3:6] = np.cross(e, c1 - A), e
    T[6:9], T[9:12] = vP + w3r * np.cross(e, c2 - P), w3r * e
    T[12:15], T[15:18] = w4r * np.cross(e, c3 - D), w4r * e
    return T[:, None]


@pytest.mark.parametrize("seed", range(5))
def test_fourbar_step_is_projection_on_loop_velocities(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.fourbar_world(rng, with_box=False)
    T = fourbar_velocity_basis(s)
    s.u = (rng.normal() * T[:, 0]).reshape(3, 6)
    dt, g = 1e-3, (0.0, 0.0, -9.81)
    P = orc.Params(dt=dt, baumgarte=0.0, eta=1e-6, rho_bil=1e-6, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    M, h = forces(s, g)
    uf = s.u.reshape(-1) + dt * np.linalg.solve(M, h)
    expected = T @ np.linalg.solve(T.T @ M @ T, T.T @ M @ uf)
    assert np.abs(out["u"].reshape(-1) - expected).max() < 1e-9 * max(1.0, np.abs(expected).max())


@pytest.mark.parametrize("theta", [0.2, 0.45])
@pytest.mark.parametrize("regime", ["stick", "slide"])
def test_box_on_incline(orc, theta, regime):
    mu = math.tan(theta) + (0.05 if regime == "stick" else -0.05)
    dt, g0, m = 1e-3, 9.81, 1.0
    s = scenes.box_on_incline(theta, mu, mass=m, dt=dt, g=g0)
    P = orc.Params(dt=dt, baumgarte=0.0, eta=1e-8, rho_bil=1e-8, rho_c=1.0, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    lam = out["lam"].reshape(4, 3)
    downhill = np.array([math.cos(theta), 0.0, -math.sin(theta)])
    n = np.array([math.sin(theta), 0.0, math.cos(theta)])
    gvec = np.array([0.0, 0.0, -g0])
    if regime == "stick":
        assert np.abs(out["u"]).max() < 1e-9
        imp = S["J"].T @ out["lam"]
        assert np.abs(imp[:3] + dt * m * gvec).max() < 1e-9
    else:
        v_exp = dt * g0 * (math.sin(theta) - mu * math.cos(theta)) * downhill
        assert np.abs(out["u"][0, :3] - v_exp).max() < 1e-9
        assert np.abs(out["u"][0, 3:]).max() < 1e-9
        assert abs(out["u"][0, :3] @ n) < 1e-12  # no normal velocity while sliding
        # every loaded contact on the cone boundary, friction opposing the slide
        t1, t2 = orc.tangent_basis(n)
        for k in range(4):
            ln, lt = lam[k, 0], lam[k, 1:]
            if ln > 1e-9:
                assert abs(np.hypot(*lt) - mu * ln) < 1e-9
                f = lt[0] * t1 + lt[1] * t2
                assert f @ downhill < 0
                assert np.linalg.norm(np.cross(f, downhill)) < 1e-9


# ---------------------------------------------------------------------------
# cross-checks that do not use PADMM
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("seed", range(4))
def test_bilateral_step_matches_dense_kkt(orc, seed):
    """Eq. 2 with R = 0: [M J^T; J 0][u+; -lambda] = [M u- + dt h; -v*]."""
    rng = np.random.default_rng(seed)
    s = scenes.random_chain_world(rng, n_bodies=4, with_limits=False, on_manifold=True)
    s.q[:, :3] += rng.normal(0.0, 1e-3, (4, 3))  # small violation: nonzero Baumgarte bias
    dt, g = 1e-3, (0.0, 0.0, -9.81)
    P = orc.Params(dt=dt, baumgarte=0.2, eta=1e-9, rho_bil=1e-9, eps=1e-11, max_iters=200000)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    J, vstar = S["J"], S["vstar"]
    M, h = forces(s, g)
    m, n = J.shape
    K = np.block([[M, J.T], [J, np.zeros((m, m))]])
    rhs = np.concatenate([M @ s.u.reshape(-1) + dt * h, -vstar])
    sol = np.linalg.solve(K, rhs)
    assert np.abs(out["u"].reshape(-1) - sol[:n]).max() < 1e-9 * max(1.0, np.abs(sol[:n]).max())
    assert np.abs(out["lam"] + sol[n:]).max() < 1e-8 * max(1.0, np.abs(sol[n:]).max())


@pytest.mark.parametrize("seed", range(4))
def test_redundant_loop_converges_to_minimum_norm_impulse(orc, seed):
    """Cold-started PADMM keeps its iterates in range(D~) when v~_f is in
    it, so its limit is the minimum-norm solution -pinv(D~) v~_f."""
    rng = np.random.default_rng(seed)
    s = scenes.fourbar_world(rng, with_box=False)
    T = fourbar_velocity_basis(s)
    s.u = (rng.normal() * T[:, 0]).reshape(3, 6) + rng.normal(0, 0.05, (3, 6))
    P = orc.Params(dt=1e-3, baumgarte=0.0, eta=1e-3, rho_bil=1e-3, eps=1e-12, max_iters=200000)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    D, vf = S["D"], S["vf"]
    p = 1.0 / np.sqrt(np.diag(D))
    Dt = p[:, None] * D * p[None, :]
    lt = -np.linalg.pinv(Dt, rcond=1e-10) @ (p * vf)
    assert np.abs(out["lam_tilde"] - lt).max() < 1e-7 * max(1.0, np.abs(lt).max())
    # and the velocity update agrees with a least-squares KKT solve
    M, h = forces(s, (0.0, 0.0, -9.81))
    J = S["J"]
    n = J.shape[1]
    K = np.block([[M, J.T], [J, np.zeros((J.shape[0], J.shape[0]))]])
    rhs = np.concatenate([M @ s.u.reshape(-1) + 1e-3 * h, -S["vstar"]])
    sol = np.linalg.lstsq(K, rhs, rcond=1e-12)[0]
    assert np.abs(out["u"].reshape(-1) - sol[:n]).max() < 1e-8


@pytest.mark.parametrize("seed", range(8))
def test_frictionless_contacts_match_lcp_enumeration(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.box_point_contacts(rng, n_points=3, mu=0.0, gap_scale=2e-3, v_scale=0.3)
    P = orc.Params(dt=1e-3, baumgarte=0.2, rho_c=1.0, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    D, vf = S["D"], S["vf"]
    nrm = np.arange(0, 9, 3)
    Dn, vn = D[np.ix_(nrm, nrm)], vf[nrm]
    sols = []
    for mask in range(8):
        act = [k for k in range(3) if mask >> k & 1]
        lam = np.zeros(3)
        if act:
            lam[act] = np.linalg.solve(Dn[np.ix_(act, act)], -vn[act])
        v = Dn @ lam + vn
        if np.all(lam >= -1e-12) and np.all(v >= -1e-12):
            sols.append(lam)
    assert len(sols) == 1
    assert np.abs(out["lam"][nrm] - sols[0]).max() < 1e-9 * max(1.0, np.abs(sols[0]).max())
    assert np.abs(np.delete(out["lam"], nrm)).max() == 0.0


def one_contact_modes(D, vf, mu):
    """All solutions of the single-contact De Saxce NCP (Eq. 3): separating,
    sticking, and sliding (lambda on the cone boundary opposing the slip
    direction phi, zero normal velocity), the last found by a scan over phi
    followed by root refinement."""
    sols = []
    if vf[0] >= 0.0:
        sols.append(np.zeros(3))
    lam = np.linalg.solve(D, -vf)
    if np.hypot(lam[1], lam[2]) <= mu * lam[0]:
        sols.append(lam)

    def resid(phi):
        d = np.array([1.0, -mu * math.cos(phi), -mu * math.sin(phi)])
        ln = -vf[0] / (D[0] @ d)
        vt = ln * (D[1:] @ d) + vf[1:]
        return math.cos(phi) * vt[1] - math.sin(phi) * vt[0], ln, vt

    grid = np.linspace(0.0, 2 * math.pi, 7201)
    vals = [resid(p)[0] for p in grid]
    for i in range(len(grid) - 1):
        if vals[i] == 0.0 or vals[i] * vals[i + 1] < 0.0:
            phi = brentq(lambda p: resid(p)[0], grid[i], grid[i + 1], xtol=1e-15) if vals[i] != 0.0 else grid[i]
            _, ln, vt = resid(phi)
            if ln > 0.0 and vt @ np.array([math.cos(phi), math.sin(phi)]) > 0.0:
                sols.append(ln * np.array([1.0, -mu * math.cos(phi), -mu * math.sin(phi)]))
    return sols


@pytest.mark.parametrize("seed", range(10))
def test_single_frictional_contact_matches_mode_enumeration(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.box_point_contacts(rng, n_points=1, mu=rng.uniform(0.2, 1.0), v_scale=0.1)
    P = orc.Params(dt=1e-3, baumgarte=0.2, rho_c=1.0, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    sols = one_contact_modes(S["D"], S["vf"], s.contact_mu[0])
    assert len(sols) >= 1
    err = min(np.abs(out["lam"] - x).max() for x in sols)
    assert err < 1e-8 * max(1.0, np.abs(out["lam"]).max())


def ncp_violation(lam, v, kind, mu):
    """Max violation of lambda in K, v + Gamma(v) in K*, and complementarity."""
    worst = 0.0
    i = 0
    while i < len(lam):
        if kind[i] == 2:
            l, w = lam[i:i + 3], v[i:i + 3].copy()
            w[0] += mu[i] * np.hypot(w[1], w[2])
            worst = max(worst, np.hypot(l[1], l[2]) - mu[i] * l[0], mu[i] * np.hypot(w[1], w[2]) - w[0],
                        abs(l @ w))
            i += 3
        elif kind[i] == 1:
            worst = max(worst, -lam[i], -v[i], abs(lam[i] * v[i]))
            i += 1
        else:
            worst = max(worst, abs(v[i]))
            i += 1
    return worst


@pytest.mark.parametrize("seed", range(6))
def test_returned_impulses_solve_the_ncp(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.box_point_contacts(rng, n_points=4, mu=rng.uniform(0.3, 1.0), gap_scale=1e-3, v_scale=0.3)
    P = orc.Params(dt=1e-3, **TIGHT, precond=int(seed % 2))
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    S = orc.world_system(s, P, 0)
    v = S["D"] @ out["lam"] + S["vf"]
    assert ncp_violation(out["lam"], v, S["kind"], S["mu"]) < 1e-10
    assert out["resid"][0, 3] < 1e-10


# ---------------------------------------------------------------------------
# solver mechanics
# ---------------------------------------------------------------------------


def test_exact_warm_start_is_a_fixed_point(orc):
    s = scenes.biped_batch(1)
    P = orc.Params(dt=2e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-9, max_iters=200000)
    cold = orc.step(s, P)
    assert cold["status"][0] == orc.OK and cold["iters"][0] > 5
    warm = orc.step(s, P, lambda_ws=cold["lam"])
    assert warm["iters"][0] == 1
    assert np.abs(warm["u"] - cold["u"]).max() < 1e-7  # one more step inside the eps ball


def test_restart_replay_reproduces_the_run(orc):
    s = scenes.fourbar_batch(6, seed=3)
    P = orc.Params(dt=1e-3, eta=1e-4, rho_bil=1e-6, rho_c=1.0, fixed_iters=50)
    a = orc.step(s, P, log_iters=50)
    assert a["restart_log"].sum() > 0
    b = orc.step(s, P, replay_log=a["restart_log"])
    assert np.array_equal(a["lam"], b["lam"]) and np.array_equal(a["u"], b["u"])
    # forcing a different schedule changes the iterates
    c = orc.step(s, P, replay_log=1 - a["restart_log"])
    assert not np.array_equal(a["lam"], c["lam"])


def test_status_flags(orc):
    s = scenes.biped_batch(2)
    P = orc.Params(dt=2e-3)
    out = orc.step(s, P.replace(max_iters=1))
    assert np.all(out["status"] == orc.MAXITER) and np.all(out["iters"] == 1)
    out = orc.step(s, P.replace(rho_bil=-1.0, eta=0.0))
    assert np.all(out["status"] & orc.FACTOR_FAIL)
    assert np.all(out["lam"] == 0.0)
    q = s.q.copy()
    q[31, 0] = np.nan  # a body of world 1
    out = orc.step(s, P, q=q)
    assert out["status"][0] == orc.OK and out["status"][1] != orc.OK
    # a corrupted world leaves the other bitwise unaffected
    ref = orc.step(s, P)
    nb0 = 31
    assert np.array_equal(out["u"][:nb0], ref["u"][:nb0])


def test_redundant_loops_with_rounded_frames_have_a_dual_residual_floor(orc):
    """Reading of the paper's redundant loops: the excavator assembled in
    FP64 converges to 1e-6 within a few tens of iterations; the same
    excavator with every input rounded to FP32 cannot close its four planar
    loops exactly, and Baumgarte feedback on the redundant rows leaves the
    dual residual a floor above 1e-6, so the cap is reached; without the
    feedback the rounded system converges again."""
    ex = scenes.excavator_batch(2, seed=1003)
    P = orc.Params(dt=2e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-6, max_iters=2000, baumgarte=0.2)
    assert np.all(orc.step(ex, P)["iters"] < 100)
    r = orc.step(scenes.round_to_f32(ex), P)
    assert np.all(r["iters"] == 2000) and np.all(r["resid"][:, 1] > 1e-6)
    assert np.all(r["resid"][:, 0] < 1e-6)
    assert np.all(orc.step(scenes.round_to_f32(ex), P.replace(baumgarte=0.0))["iters"] < 100)
