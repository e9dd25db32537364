"""Pins of the oracle's contact generators: resting and stacked boxes with
closed-form contact sets, a corner pushed into the floor, the deepest-first
cap, and probe contacts."""
import numpy as np

from oracle import contacts as OC
from paper_2603_16536_amd import scenes

I3 = np.eye(3)


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def test_cube_resting_on_the_floor():
    h = np.array([0.05, 0.05, 0.05])
    got = OC.box_bin_world([np.array([0.0, 0.0, 0.05])], [I3], [h], [0.7], 0.15, 0.15, 0.01, 64)
    assert len(got) == 4
    for x in got:
        assert x["target"] == 0 and x["gap"] == 0.0 and np.array_equal(x["normal"], [0, 0, 1])
        assert abs(abs(x["point"][0]) - 0.05) < 1e-15 and x["point"][2] == 0.0
        assert x["mu"] == 0.7
    assert sorted(x["key"] & 7 for x in got) == [0, 1, 2, 3]  # the four -z vertices


def test_small_cube_stacked_on_a_large_one():
    """The upper cube's four bottom vertices sit on the lower cube's top face
    (gap 0, normal +z from the lower to the upper cube); the lower cube's top
    vertices lie outside the upper cube's faces' extent (no contact); the
    lower cube's bottom vertices touch the floor."""
    hl, hs = np.array([0.05] * 3), np.array([0.03] * 3)
    c = [np.array([0.0, 0.0, 0.05]), np.array([0.0, 0.0, 0.13])]
    got = OC.box_bin_world(c, [I3, I3], [hl, hs], [0.9, 0.4], 0.15, 0.15, 0.01, 64)
    floor = [x for x in got if x["target"] == 0]
    box = [x for x in got if x["target"] >= 5]
    assert len(floor) == 4 and all(x["box"] == 0 for x in floor)
    assert len(box) == 4
    for x in box:
        assert x["box"] == 1 and x["target"] == 5 and abs(x["gap"]) < 1e-15
        assert np.allclose(x["normal"], [0, 0, 1]) and x["mu"] == 0.4
        assert abs(x["point"][2] - 0.10) < 1e-15


def test_tilted_box_corner_penetrates_the_floor():
    """A 0.08 x 0.04 x 0.02 box rotated 30 degrees about y with its lowest
    edge 2 mm deep: the two vertices of that edge at gap -0.002, the two of
    the edge above it at 2 hz cos 30 - 0.002 (inside the 2 cm margin), the
    rest 2 hx sin 30 higher (outside)."""
    h = np.array([0.04, 0.02, 0.01])
    a = np.deg2rad(30.0)
    R = rot_y(a)
    c = np.array([0.0, 0.0, h[0] * np.sin(a) + h[2] * np.cos(a) - 0.002])
    got = OC.box_bin_world([c], [R], [h], [0.5], 0.15, 0.15, 0.02, 64)
    gaps = sorted(x["gap"] for x in got)
    assert all(x["target"] == 0 for x in got) and len(gaps) == 4
    assert np.allclose(gaps[:2], -0.002, atol=1e-15)
    assert np.allclose(gaps[2:], 2 * h[2] * np.cos(a) - 0.002, atol=1e-15)


def test_cap_keeps_the_deepest_with_key_order_on_ties():
    h = np.array([0.05, 0.05, 0.05])
    c = [np.array([x, 0.0, 0.05 - 0.001 * i]) for i, x in enumerate([-0.09, 0.0, 0.09])]
    got = OC.box_bin_world(c, [I3] * 3, [h] * 3, [0.5] * 3, 0.15, 0.15, 0.01, 6)
    assert len(got) == 6
    g = [x["gap"] for x in got]
    assert g == sorted(g)
    # the deepest box (third, -2 mm) first, its four floor vertices by key
    assert [x["box"] for x in got[:4]] == [2, 2, 2, 2]
    assert [x["key"] for x in got[:4]] == sorted(x["key"] for x in got[:4])


def test_walls_have_inward_normals():
    h = np.array([0.02, 0.02, 0.02])
    got = OC.box_bin_world([np.array([0.131, -0.131, 0.3])], [I3], [h], [0.5], 0.15, 0.15, 0.01, 64)
    by_t = {}
    for x in got:
        by_t.setdefault(x["target"], []).append(x)
    assert set(by_t) == {2, 3}  # wall +x and wall -y
    for x in by_t[2]:
        assert np.array_equal(x["normal"], [-1, 0, 0]) and abs(x["gap"] - (0.15 - 0.151)) < 1e-12
    for x in by_t[3]:
        assert np.array_equal(x["normal"], [0, 1, 0]) and abs(x["gap"] - (-0.151 + 0.15)) < 1e-12


def test_probe_contacts_of_the_standing_biped():
    bp = scenes.biped_batch(2)
    sc = OC.probe_contacts(bp, bp.q, 0.02)
    assert sc.n_contacts == 16
    assert np.all(sc.contact_key[:8] == np.arange(8))
    assert np.abs(sc.contact_gap).max() < 1e-12


def test_generated_box_bin_worlds_start_apart():
    bb = scenes.box_bin_batch(4, seed=9)
    assert bb.n_bodies == 80 and bb.body_box.shape == (80, 4)
    cap = 64
    sc = OC.box_bin_contacts(bb, bb.q, 0.15, 0.15, 0.0, cap)
    assert sc.n_contacts == 0  # nothing touches at the start
    m = bb.body_mass
    assert m.min() > 0 and m.max() / m.min() > 10
