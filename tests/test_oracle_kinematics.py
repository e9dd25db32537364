"""Pins of the oracle's kinematics (Sec. 3): constraint Jacobians against
central finite differences of the position-level constraint functions,
contact rows against finite differences of material-point positions, the
tangent basis against its definition, and the scene generators' poses
against the constraint manifold and Freudenstein's four-bar equation."""
import math

import numpy as np
import pytest

from paper_2603_16536_amd import scenes


def qmul(p, q):
    return np.array([
        p[3] * q[0] + p[0] * q[3] + p[1] * q[2] - p[2] * q[1],
        p[3] * q[1] - p[0] * q[2] + p[1] * q[3] + p[2] * q[0],
        p[3] * q[2] + p[0] * q[1] - p[1] * q[0] + p[2] * q[3],
        p[3] * q[3] - p[0] * q[0] - p[1] * q[1] - p[2] * q[2],
    ])


def perturb(q, body, k, eps):
    """Move body along generalized velocity direction k (v_x..v_z, w_x..w_z,
    world frame) by eps: translation, or left multiplication by exp(eps e)."""
    q = q.copy()
    if k < 3:
        q[body, k] += eps
    else:
        axis = np.zeros(3)
        axis[k - 3] = 1.0
        dq = np.concatenate([axis * math.sin(0.5 * eps), [math.cos(0.5 * eps)]])
        q[body, 3:] = qmul(dq, q[body, 3:])
    return q


def fd_jacobian(orc, scene, params, w, rows, eps=1e-6):
    nb, _ = orc.world_dims(scene, w)
    b0 = scene.body_offsets()[w]
    J = np.zeros((len(rows), 6 * nb))
    for i in range(nb):
        for k in range(6):
            fp = orc.world_system(scene, params, w, q=perturb(scene.q, b0 + i, k, eps))["f"]
            fm = orc.world_system(scene, params, w, q=perturb(scene.q, b0 + i, k, -eps))["f"]
            J[:, 6 * i + k] = (fp[rows] - fm[rows]) / (2 * eps)
    return J


@pytest.mark.parametrize("seed", range(6))
def test_joint_and_limit_jacobians_match_finite_differences(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.random_chain_world(rng, n_bodies=4, with_limits=True)
    P = orc.Params()
    S = orc.world_system(s, P, 0)
    rows = np.where(S["kind"] <= orc.ROW_LIMIT)[0]
    Jfd = fd_jacobian(orc, s, P, 0, rows)
    # revolute limit rows are exact only for aligned axes; off the manifold
    # compare bilateral rows everywhere and limit rows of prismatic joints
    nj = s.n_joints
    limited = [j for j in range(nj) if not np.all(np.isnan(s.joint_limit[j]))]
    keep = list(range(5 * nj))
    for r, j in enumerate(limited):
        if s.joint_type[j] == scenes.PRISMATIC:
            keep.append(5 * nj + r)
    keep = np.array(keep)
    err = np.abs(S["J"][keep] - Jfd[keep]).max()
    assert err < 1e-7 * max(1.0, np.abs(Jfd).max()), err


@pytest.mark.parametrize("seed", range(4))
def test_limit_rows_on_manifold_match_finite_differences(orc, seed):
    rng = np.random.default_rng(100 + seed)
    s = scenes.random_chain_world(rng, n_bodies=3, with_limits=True, on_manifold=True)
    P = orc.Params()
    S = orc.world_system(s, P, 0)
    assert np.abs(S["f"][S["kind"] == orc.ROW_BILATERAL]).max() < 1e-12
    rows = np.where(S["kind"] <= orc.ROW_LIMIT)[0]
    Jfd = fd_jacobian(orc, s, P, 0, rows)
    assert np.abs(S["J"][rows] - Jfd).max() < 1e-7


@pytest.mark.parametrize("seed", range(4))
def test_joint_coordinate_jacobian(orc, seed):
    rng = np.random.default_rng(200 + seed)
    s = scenes.random_chain_world(rng, n_bodies=3, with_limits=False, on_manifold=True)
    eps = 1e-6
    for j in range(s.n_joints):
        c, Ja, Jb = orc.joint_coordinate(s, s.q, j)
        a, b = s.joint_body[j]
        for body, Jside in ((a, Ja), (b, Jb)):
            if body < 0:
                continue
            for k in range(6):
                cp = orc.joint_coordinate(s, perturb(s.q, body, k, eps), j)[0]
                cm = orc.joint_coordinate(s, perturb(s.q, body, k, -eps), j)[0]
                assert abs((cp - cm) / (2 * eps) - Jside[k]) < 1e-7


def test_contact_rows_are_material_point_velocities(orc):
    """A contact row, applied to the twists, is the finite-difference rate of
    d . (x_a - x_b) where x_a, x_b are the material points of the two bodies
    that coincide with the contact point."""
    rng = np.random.default_rng(7)
    s = scenes.random_chain_world(rng, n_bodies=2, with_limits=False)
    # add a contact between body 1 and body 0 and one against the ground
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    p = rng.normal(0, 0.3, 3)
    s = s.replace(contact_world=np.zeros(2, np.int32), contact_body=np.array([[1, 0], [0, -1]], np.int32),
                  contact_point=np.stack([p, p + 0.1]), contact_normal=np.stack([n, n]),
                  contact_gap=np.zeros(2), contact_mu=np.full(2, 0.5), contact_key=np.arange(2, dtype=np.int32))
    P = orc.Params()
    S = orc.world_system(s, P, 0)
    crow = np.where(S["kind"] >= orc.ROW_NORMAL)[0]
    t1, t2 = orc.tangent_basis(n)
    dirs = [n, t1, t2]
    eps = 1e-6
    q0 = s.q

    def rot(q):
        x, y, z, w = q
        return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                         [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                         [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])

    def material(q, body, point):
        if body < 0:
            return point
        loc = rot(q0[body, 3:]).T @ (point - q0[body, :3])
        return q[body, :3] + rot(q[body, 3:]) @ loc

    for c in range(2):
        a, b = s.contact_body[c]
        point = s.contact_point[c]
        for e in range(3):
            r = crow[3 * c + e]
            for body in range(2):
                for k in range(6):
                    qp, qm = perturb(q0, body, k, eps), perturb(q0, body, k, -eps)
                    gp = dirs[e] @ (material(qp, a, point) - material(qp, b, point))
                    gm = dirs[e] @ (material(qm, a, point) - material(qm, b, point))
                    assert abs((gp - gm) / (2 * eps) - S["J"][r, 6 * body + k]) < 1e-7


def test_tangent_basis_is_orthonormal_and_right_handed(orc):
    rng = np.random.default_rng(3)
    normals = list(rng.normal(size=(50, 3))) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0]),
                                                 np.array([1.0, 0, 0]), np.array([0, 1.0, 0])]
    for n in normals:
        n = n / np.linalg.norm(n)
        t1, t2 = orc.tangent_basis(n)
        B = np.stack([n, t1, t2])
        assert np.abs(B @ B.T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(np.stack([t1, t2, n])) - 1.0) < 1e-14


def test_generated_worlds_lie_on_the_constraint_manifold(orc):
    P = orc.Params()
    fb = scenes.fourbar_batch(8, seed=5)
    for w in range(8):
        S = orc.world_system(fb, P, w)
        assert np.abs(S["f"][S["kind"] == orc.ROW_BILATERAL]).max() < 1e-14
        assert np.linalg.matrix_rank(S["J"][:20], tol=1e-9) == 17  # planar RRRR loop: 3 redundant rows
    bp = scenes.biped_batch(1)
    S = orc.world_system(bp, orc.Params(dt=2e-3), 0)
    assert S["J"].shape == (224, 186)
    assert np.abs(S["f"][S["kind"] == orc.ROW_BILATERAL]).max() < 1e-14
    # ten planar parallelogram loops, three redundant rows each
    assert np.linalg.matrix_rank(S["J"][:200], tol=1e-9) == 170


def test_fourbar_geometry_satisfies_freudenstein():
    """Freudenstein's equation for pivots at (0, 0) and (d, 0):
    (d/a) cos th4 - (d/c) cos th2 + (a^2 - b^2 + c^2 + d^2)/(2 a c) = cos(th2 - th4)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        g = scenes.fourbar_geometry(rng)
        a, b, c, d = g["a"], g["b"], g["c"], g["d"]
        th2 = math.atan2(g["P"][1], g["P"][0])
        th4 = math.atan2(g["Q"][1] - g["D"][1], g["Q"][0] - g["D"][0])
        lhs = (d / a) * math.cos(th4) - (d / c) * math.cos(th2) + (a * a - b * b + c * c + d * d) / (2 * a * c)
        assert abs(lhs - math.cos(th2 - th4)) < 1e-12
        assert abs(th2 - g["th2"]) < 1e-12


def test_excavator_assembly_and_mobility(orc):
    """The hydraulic excavator is assembled on the manifold; its four planar
    loops leave 80 - 12 = 68 independent bilateral rows, i.e. four degrees
    of freedom (swing and the three cylinder strokes, Gruebler count
    72 - 68); the three stroke-limit rows sit at the nearer bound, 0.35 m
    away, and with them the mechanism keeps only the swing."""
    ex = scenes.excavator_batch(4, seed=9)
    assert ex.n_bodies == 48 and ex.n_joints == 64
    for w in range(4):
        S = orc.world_system(ex, orc.Params(dt=2e-3), w)
        bil = S["kind"] == orc.ROW_BILATERAL
        assert S["J"].shape == (83, 72) and bil.sum() == 80
        assert np.abs(S["f"][bil]).max() < 1e-12
        assert np.linalg.matrix_rank(S["J"][bil], tol=1e-9) == 68
        assert np.allclose(S["f"][S["kind"] == orc.ROW_LIMIT], 0.35, atol=1e-12)
        assert np.linalg.matrix_rank(S["J"], tol=1e-9) == 71
    m = ex.body_mass[:12]
    assert m.max() / m.min() == pytest.approx(1e4)


def test_heterogeneous_batch_interleaves_three_structures():
    h = scenes.heterogeneous_batch(7, seed=3)
    nb = np.diff(h.body_offsets())
    assert nb.tolist() == [4, 31, 12, 4, 31, 12, 4]
    nj = np.diff(h.joint_offsets())
    assert nj.tolist() == [4, 40, 16, 4, 40, 16, 4]
