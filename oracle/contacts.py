"""FP64 contact generation for the oracle side.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU
leg.  Contacts are inputs of the step (Sec. 3: point, normal from body b to
body a, signed gap, friction); these generators produce them from the state
independently of the device's own generation, so that no oracle input is
read back from the device.

* probes: body-fixed points tested against the plane z = 0; a probe whose
  height is below the margin becomes a contact with normal +z and gap equal
  to the height, key = the probe's index within its world, in probe order.
* boxes in a bin: every vertex of every box against the floor z = 0, the
  walls x = -wx, x = +wx, y = -wy, y = +wy (targets 0-4) and the faces of
  every other box of the world (target 5 + k).  Against a box the vertex is
  taken to the box frame; with d_e = |q_e| - h_e the face is the axis of the
  largest d_e, the gap is that d_e, and the vertex must lie over the face
  (the other two d_e <= 0).  The normal is the outward face normal (from the
  target to the vertex's box).  Kept: gap < margin; of those the deepest
  first, ties by key = (target * 64 + box) * 8 + vertex, at most ``cap``.
"""
from __future__ import annotations

import numpy as np

MAX_BODIES = 64
_PLANE_NORMALS = np.array([[0, 0, 1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0]], np.float64)


def _rot(q):
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def probe_contacts(scene, q, margin):
    """The scene with explicit contacts from its probes at poses q."""
    cw, cb, cp, cg, cm, ck = [], [], [], [], [], []
    po = scene.probe_offsets()
    for w in range(scene.n_worlds):
        for k in range(po[w], po[w + 1]):
            b = scene.probe_body[k]
            pw = q[b, :3] + _rot(q[b, 3:]) @ scene.probe_point[k]
            if pw[2] < margin:
                cw.append(w)
                cb.append((b, -1))
                cp.append(pw)
                cg.append(pw[2])
                cm.append(scene.probe_mu[k])
                ck.append(k - po[w])
    n = len(cw)
    return scene.replace(contact_world=np.array(cw, np.int32), contact_body=np.array(cb, np.int32).reshape(n, 2),
                         contact_point=np.array(cp).reshape(n, 3), contact_normal=np.tile([0.0, 0.0, 1.0], (n, 1)),
                         contact_gap=np.array(cg), contact_mu=np.array(cm), contact_key=np.array(ck, np.int32))


def _vertices(c, R, h):
    s = np.array([[(v >> e) & 1 for e in range(3)] for v in range(8)], np.float64) * 2 - 1
    return c + (s * h) @ R.T


def box_candidates(c_list, R_list, h_list, wx, wy):
    """Every (key, gap, normal, point, box, target) of one world, before the
    margin test.  Also returns, per candidate, the smallest distance of a
    decision quantity to its threshold (lateral extents and face choice),
    so callers can recognise decisions that rounding could flip."""
    n = len(c_list)
    out = []
    for k in range(n):
        V = _vertices(c_list[k], R_list[k], h_list[k])
        for v in range(8):
            p = V[v]
            for t in range(5 + n):
                if t >= 5 and t - 5 == k:
                    continue
                if t < 5:
                    gap = [p[2], p[0] + wx, wx - p[0], p[1] + wy, wy - p[1]][t]
                    nrm = _PLANE_NORMALS[t]
                    slack = np.inf
                else:
                    j = t - 5
                    qv = R_list[j].T @ (p - c_list[j])
                    d = np.abs(qv) - h_list[j]
                    f = int(np.argmax(d))
                    others = [e for e in range(3) if e != f]
                    slack = min(min(abs(d[e]) for e in others), d[f] - max(d[e] for e in others))
                    if any(d[e] > 0.0 for e in others):
                        out.append(dict(key=(t * MAX_BODIES + k) * 8 + v, gap=None, slack=slack))
                        continue
                    gap = d[f]
                    nrm = np.sign(qv[f]) * R_list[j][:, f] if qv[f] != 0 else R_list[j][:, f]
                out.append(dict(key=(t * MAX_BODIES + k) * 8 + v, gap=float(gap), normal=np.asarray(nrm, np.float64),
                                point=p.copy(), box=k, target=t, slack=slack))
    return out


def box_bin_world(c_list, R_list, h_list, mu_list, wx, wy, margin, cap):
    """Contacts of one world (list of dicts, deepest first)."""
    cands = [x for x in box_candidates(c_list, R_list, h_list, wx, wy) if x["gap"] is not None and x["gap"] < margin]
    cands.sort(key=lambda x: (x["gap"], x["key"]))
    kept = cands[:cap]
    for x in kept:
        t = x["target"]
        x["mu"] = mu_list[x["box"]] if t < 5 else min(mu_list[x["box"]], mu_list[t - 5])
    return kept


def box_bin_contacts(scene, q, wx, wy, margin, cap):
    """The scene with explicit contacts from box-in-bin tests at poses q
    (boxes: bodies with positive ``scene.body_box`` half extents)."""
    cw, cb, cp, cn, cg, cm, ck = [], [], [], [], [], [], []
    bo = scene.body_offsets()
    for w in range(scene.n_worlds):
        boxes = [b for b in range(bo[w], bo[w + 1]) if scene.body_box[b, 0] > 0]
        c_list = [q[b, :3] for b in boxes]
        R_list = [_rot(q[b, 3:]) for b in boxes]
        h_list = [scene.body_box[b, :3] for b in boxes]
        mu_list = [scene.body_box[b, 3] for b in boxes]
        for x in box_bin_world(c_list, R_list, h_list, mu_list, wx, wy, margin, cap):
            t = x["target"]
            cw.append(w)
            cb.append((boxes[x["box"]], -1 if t < 5 else boxes[t - 5]))
            cp.append(x["point"])
            cn.append(x["normal"])
            cg.append(x["gap"])
            cm.append(x["mu"])
            ck.append(x["key"])
    n = len(cw)
    return scene.replace(contact_world=np.array(cw, np.int32), contact_body=np.array(cb, np.int32).reshape(n, 2),
                         contact_point=np.array(cp).reshape(n, 3), contact_normal=np.array(cn).reshape(n, 3),
                         contact_gap=np.array(cg), contact_mu=np.array(cm), contact_key=np.array(ck, np.int32))
