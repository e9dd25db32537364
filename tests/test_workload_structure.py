"""Loop structure of the synthetic workloads.

Independent closed kinematic chains are the cyclomatic number of the joint
graph (bodies and the world as nodes, joints as edges): E - V + C.  The count
is pinned against the paper's own systems table (Sec. 6.1, Tab. 1;
`golden/systems_tab1.txt`), then used to check that every seeded generator
builds the topology its workload recipe states (joints, bodies, loops)."""
import os

import numpy as np
import pytest

from paper_2603_16536_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))


def read_tab1():
    rows = []
    for line in open(os.path.join(HERE, "golden", "systems_tab1.txt")):
        line = line.split("#", 1)[0].split()
        if line:
            name, nb, na, npas, loops, base = line
            rows.append((name, int(nb), int(na), int(npas), int(loops), base))
    return rows


def cyclomatic(n_nodes, edges):
    """E - V + C of an undirected multigraph (union-find over the nodes)."""
    parent = list(range(n_nodes))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[ra] = rb
    comps = len({find(a) for a in range(n_nodes)})
    return len(edges) - n_nodes + comps


def world_topology(scene, w):
    """(bodies, joints by type, loops) of world w; node 0 is the fixed world."""
    bo, jo = scene.body_offsets(), scene.joint_offsets()
    b0, b1, j0, j1 = bo[w], bo[w + 1], jo[w], jo[w + 1]
    edges = []
    for a, b in scene.joint_body[j0:j1]:
        edges.append((0 if a < 0 else a - b0 + 1, 0 if b < 0 else b - b0 + 1))
    types = np.bincount(scene.joint_type[j0:j1], minlength=2)
    return b1 - b0, types, cyclomatic(b1 - b0 + 1, edges)


def test_cyclomatic_number_reproduces_the_paper_table():
    rows = read_tab1()
    assert [r[0] for r in rows] == ["DR_Legs", "BDX", "Olaf", "Iron_Man"]
    for name, nb, na, npas, loops, base in rows:
        joints = na + npas
        if base == "tree":
            assert loops == 0, name
            continue
        # one connected system: the world joins as a node only when a joint reaches it
        nodes = nb + (1 if base == "fixed" else 0)
        assert joints - nodes + 1 == loops, name


def test_cyclomatic_number_on_small_graphs():
    assert cyclomatic(4, [(0, 1), (1, 2), (2, 3), (3, 0)]) == 1       # one ring
    assert cyclomatic(5, [(0, 1), (1, 2), (2, 3), (3, 0)]) == 1       # plus an isolated node
    assert cyclomatic(3, [(0, 1), (0, 1), (1, 2)]) == 1               # parallel joints close a loop
    assert cyclomatic(6, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3)]) == 2
    assert cyclomatic(4, [(0, 1), (1, 2), (2, 3)]) == 0               # a chain


@pytest.mark.parametrize("make,bodies,revolute,prismatic,loops", [
    (lambda: scenes.fourbar_batch(8, seed=1001), 4, 4, 0, 1),        # three links + cube, ground = world
    (lambda: scenes.free_fourbar_batch(8, seed=1006), 4, 4, 0, 1),
    (lambda: scenes.biped_batch(8, seed=1002), 31, 40, 0, 10),
    (lambda: scenes.excavator_batch(8, seed=1003), 12, 13, 3, 4),
    (lambda: scenes.box_bin_batch(4, seed=1005), 20, 0, 0, 0),
    (lambda: scenes.figure_batch(2, seed=1007), 151, 196, 0, 45),
])
def test_generators_build_the_stated_topology(make, bodies, revolute, prismatic, loops):
    scene = make()
    for w in range(scene.n_worlds):
        nb, types, cyc = world_topology(scene, w)
        assert (nb, int(types[scenes.REVOLUTE]), int(types[scenes.PRISMATIC]), cyc) == \
            (bodies, revolute, prismatic, loops), w


def test_heterogeneous_batch_mixes_the_three_topologies():
    scene = scenes.heterogeneous_batch(12, seed=1003)
    seen = {world_topology(scene, w)[2] for w in range(scene.n_worlds)}
    assert seen == {1, 10, 4}


def test_fixed_figure_matches_the_largest_system_of_the_table():
    """The fixed figure has the paper's largest system's counts (Tab. 1):
    bodies, actuated and passive joints, loops, and its base on the world."""
    row = [r for r in read_tab1() if r[0] == "Iron_Man"][0]
    _, nb, na, npas, loops, base = row
    scene = scenes.figure_batch(1, seed=1007)
    got_nb, types, cyc = world_topology(scene, 0)
    assert base == "fixed" and np.any(scene.joint_body[:, 1] < 0)
    assert (got_nb, int(types.sum()), int(scene.joint_actuated.sum()), cyc) == (nb, na + npas, na, loops)


def test_fixed_figure_explicit_gains_are_stable_at_its_step():
    """An explicit PD torque on a joint whose moving side has inertia I about
    the joint axis advances omega by -(kd dt / I) omega - (kp dt^2 / I) theta
    per step: the figure's actuated joints keep kd dt / I <= 0.5 and
    kp dt^2 / I <= 0.1 against the child body's inertia about the axis,
    taken here from the kinetic energy of a unit rotation about the joint
    line (1/2 m |w x r|^2 + 1/2 w^T I_world w), and the heavy joints keep
    their nominal gains."""
    scene = scenes.figure_batch(1, seed=1007)
    dt = 2e-3
    nominal_kept = 0
    for j in np.where(scene.joint_actuated)[0]:
        child, _ = scene.joint_body[j]
        fa = scene.joint_frame[j, :7]
        Rb = scenes.quat_to_mat(scene.q[child][3:])
        point = scene.q[child][:3] + Rb @ fa[:3]
        axis = Rb @ scenes.quat_to_mat(fa[3:])[:, 0]
        r = scene.q[child][:3] - point
        v = np.cross(axis, r)
        Iw = Rb @ np.diag(scene.body_inertia[child]) @ Rb.T
        I = scene.body_mass[child] * (v @ v) + axis @ Iw @ axis
        kp, kd = scene.joint_pd[j]
        assert kd * dt / I <= 0.5 + 1e-9 and kp * dt * dt / I <= 0.1 + 1e-9, (j, kp, kd, I)
        assert kp > 0.0 and kd > 0.0
        nominal_kept += kp in (400.0, 300.0, 200.0, 100.0, 20.0)
    assert nominal_kept >= 10


def test_fixed_figure_rollout_stays_bounded(orc):
    """Two figures under their explicit PD toward the assembled pose plus
    N(0, 5 N m) torques, stepped by the oracle (exact x-updates): every step
    converges to 1e-6 in a few iterations and the twists stay bounded."""
    orc.set_threads(4)
    scene = scenes.round_to_f32(scenes.figure_batch(2, seed=1007))
    P = orc.Params(dt=2e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-6, max_iters=200, baumgarte=0.2)
    act = np.where(scene.joint_actuated)[0]
    rng = np.random.default_rng(3)
    q, u = scene.q.copy(), scene.u.copy()
    for _ in range(8):
        qr = orc.step_configuration(scene, P, q=q, u=u)
        tau = np.zeros(scene.n_joints)
        for j in act:
            kp, kd = scene.joint_pd[j]
            c, Ja, Jb = orc.joint_coordinate(scene, qr, j)
            a, b = scene.joint_body[j]
            rate = Ja @ u[a] + (Jb @ u[b] if b >= 0 else 0.0)
            tau[j] = -kp * c - kd * rate + 5.0 * rng.normal()
        o = orc.step(scene, P, q=q, u=u, joint_torque=tau)
        assert np.all(o["status"] == orc.OK) and o["iters"].max() <= 10
        q, u = o["q"], o["u"]
    assert np.abs(u).max() < 100.0


def test_rl_biped_drives_the_legs_through_the_linkages():
    """The RL stepping bipeds (Sec. 6.1, Sec. 6.3): per leg the hip yaw and
    roll keep explicit PD, hip pitch, knee and ankle are passive, and the
    five transmission cranks carry implicit PD rows with rotor armature and
    damping; the loops are unchanged and every world fits 224 rows
    (5 per revolute joint, 1 per drive, 3 per sole probe)."""
    base = scenes.round_to_f32(scenes.biped_batch(3, seed=1002, dt=4e-3, sole_probes=2))
    scene = scenes.with_drives(base, "transmission")
    jo, po = scene.joint_offsets(), scene.probe_offsets()
    for w in range(scene.n_worlds):
        js = np.arange(jo[w], jo[w + 1])
        assert world_topology(scene, w)[2] == 10
        driven = js[np.any(scene.joint_drive[js] != 0, axis=1)]
        assert len(driven) == 10
        assert np.allclose(scene.joint_drive[driven, :2], scenes.BIPED_PD)
        assert np.all(scene.joint_drive[driven, 3] > 0) and np.all(scene.joint_drive[driven, 2] > 0)
        assert np.all(scene.joint_actuated[driven] == 1)
        explicit = js[np.any(scene.joint_pd[js] != 0, axis=1)]
        assert len(explicit) == 4 and not np.intersect1d(explicit, driven).size
        assert np.count_nonzero(scene.joint_actuated[js]) == 14
        rows = 5 * len(js) + len(driven) + 3 * (po[w + 1] - po[w])
        assert rows <= 224, rows
