"""Pins of the oracle's forward kinematics (Sec. 6.3: poses consistent with
every joint, including the passive joints of kinematic loops, from target
joint coordinates, by Gauss-Newton):

* a serial chain with every joint targeted has the textbook closed form:
  the child's pose is the parent's pose times the parent-side joint frame,
  the joint's own motion (a rotation by c about x for a hinge, a
  translation by c along x for a slider) and the inverse child-side frame;
* a planar four-bar with its crank targeted puts the coupler-rocker pin on
  the intersection of the two circles about the moved crank pin and the
  fixed rocker pivot (the branch of the assembly), as Freudenstein's
  equation fixes;
* the biped: every constraint satisfied, the targets reached, the pelvis
  untouched, in a few iterations.
"""
import math

import numpy as np
import pytest

from paper_2603_16536_amd import scenes


def rot(q):
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def homog(p, q):
    T = np.eye(4)
    T[:3, :3] = rot(q)
    T[:3, 3] = p
    return T


@pytest.mark.parametrize("seed", range(4))
def test_serial_chain_matches_closed_form(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.random_chain_world(rng, n_bodies=4, with_limits=False, on_manifold=True)
    targets = rng.uniform(-0.8, 0.8, s.n_joints)
    q, iters, res = orc.forward_kinematics(s, targets, base=np.array([-1]))
    assert res[0] < 1e-12 and iters[0] < 30
    X = {-1: np.eye(4)}
    for j in range(s.n_joints):  # joint j: child body j, parent body j - 1
        a, b = s.joint_body[j]
        Fa = homog(s.joint_frame[j, :3], s.joint_frame[j, 3:7])
        Fb = homog(s.joint_frame[j, 7:10], s.joint_frame[j, 10:14])
        Mj = np.eye(4)
        c = targets[j]
        if s.joint_type[j] == scenes.REVOLUTE:
            Mj[:3, :3] = np.array([[1, 0, 0], [0, math.cos(c), -math.sin(c)], [0, math.sin(c), math.cos(c)]])
        else:
            Mj[0, 3] = c
        X[a] = X[b] @ Fb @ Mj @ np.linalg.inv(Fa)
    for i in range(s.n_bodies):
        assert np.abs(q[i, :3] - X[i][:3, 3]).max() < 1e-10
        assert np.abs(rot(q[i, 3:]) - X[i][:3, :3]).max() < 1e-10


@pytest.mark.parametrize("seed", range(4))
def test_fourbar_crank_target_follows_the_loop_closure(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.fourbar_world(rng, with_box=False)
    geo = s.meta
    O = np.array([0.0, 0.0, 0.6])
    delta = rng.uniform(-0.15, 0.15)
    targets = np.full(s.n_joints, np.nan)
    targets[0] = delta  # crank hinge, axis +y: the x-z angle atan2(z, x) of the crank decreases by delta
    q, iters, res = orc.forward_kinematics(s, targets)
    assert res[0] < 1e-12
    th2 = geo["th2"] - delta
    P = np.array([geo["a"] * math.cos(th2), geo["a"] * math.sin(th2)])
    D = geo["D"]
    e = D - P
    dist = np.linalg.norm(e)
    x = (dist * dist + geo["b"] ** 2 - geo["c"] ** 2) / (2 * dist)
    h = math.sqrt(geo["b"] ** 2 - x * x)
    ex = e / dist
    Q = P + x * ex + h * np.array([-ex[1], ex[0]])  # the assembly's branch
    # Freudenstein: K1 cos th4 - K2 cos th2 + K3 = cos(th2 - th4) with the rocker angle th4 at D
    th4 = math.atan2(Q[1] - D[1], Q[0] - D[0])
    a, b, c, d = geo["a"], geo["b"], geo["c"], geo["d"]
    K1, K2, K3 = d / a, d / c, (a * a - b * b + c * c + d * d) / (2 * a * c)
    assert abs(K1 * math.cos(th4) - K2 * math.cos(th2) + K3 - math.cos(th2 - th4)) < 1e-12
    # the rocker's far end (its rod runs from D to Q) and the crank's end P
    rocker_end = q[2, :3] + rot(q[2, 3:]) @ np.array([0.5 * c, 0.0, 0.0])
    crank_end = q[0, :3] + rot(q[0, 3:]) @ np.array([0.5 * a, 0.0, 0.0])
    assert np.abs(rocker_end - (O + np.array([Q[0], 0.0, Q[1]]))).max() < 1e-10
    assert np.abs(crank_end - (O + np.array([P[0], 0.0, P[1]]))).max() < 1e-10


def test_biped_random_targets(orc):
    s = scenes.biped_batch(4)
    rng = np.random.default_rng(11)
    targets = np.full(s.n_joints, np.nan)
    act = s.joint_actuated.astype(bool)
    targets[act] = rng.uniform(-0.3, 0.3, act.sum())
    q, iters, res = orc.forward_kinematics(s, targets)
    assert np.all(res < 1e-12) and np.all(iters <= 8)
    P = orc.Params(dt=2e-3)
    sb = s.replace(q=q)
    bo = s.body_offsets()
    for w in range(4):
        S = orc.world_system(sb, P, w)
        assert np.abs(S["f"][S["kind"] == orc.ROW_BILATERAL][:200]).max() < 1e-12
        pelvis = bo[w] + s.reset_body[w] - bo[w]
        assert np.array_equal(q[pelvis], s.q[pelvis])
    for j in np.nonzero(act)[0]:
        assert abs(orc.joint_coordinate(sb, q, j)[0] - targets[j]) < 1e-12
    # already consistent: targets at the current coordinates give no motion
    t0 = np.full(s.n_joints, np.nan)
    t0[act] = [orc.joint_coordinate(sb, q, j)[0] for j in np.nonzero(act)[0]]
    q2, it2, _ = orc.forward_kinematics(sb, t0)
    assert np.all(it2 <= 1) and np.abs(q2 - q).max() < 1e-12
