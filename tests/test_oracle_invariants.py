"""Invariants of the oracle's time step (Sec. 3: constraint impulses are
internal forces of the mechanism; the velocity update of Eq. 2 is a
projection): a closed four-bar loop floating free of the world, without
gravity, with random (inconsistent) twists.

* Linear momentum is conserved exactly: every joint applies equal and
  opposite impulses to its two bodies.
* Angular momentum about the origin is conserved exactly when the bodies
  start without spin (no gyroscopic term in the free velocity): the point
  rows act at the common anchor and the axis rows are pure couples.
* Without the Baumgarte bias the step is the M-orthogonal projection of the
  free velocity onto J u = 0: kinetic energy does not increase and the
  constraint velocities vanish.
* Over a rollout with the bias the position-level constraint violation
  stays small and does not grow.
"""
import numpy as np
import pytest

from paper_2603_16536_amd import scenes

TIGHT = dict(eps=1e-12, max_iters=200000)


def rot(q):
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def momenta(scene, q, u):
    """Total linear momentum and angular momentum about the origin."""
    p = np.zeros(3)
    L = np.zeros(3)
    for b in range(scene.n_bodies):
        m = scene.body_mass[b]
        R = rot(q[b, 3:])
        Iw = R @ np.diag(scene.body_inertia[b]) @ R.T
        p += m * u[b, :3]
        L += np.cross(q[b, :3], m * u[b, :3]) + Iw @ u[b, 3:]
    return p, L


def kinetic(scene, q, u):
    e = 0.0
    for b in range(scene.n_bodies):
        R = rot(q[b, 3:])
        Iw = R @ np.diag(scene.body_inertia[b]) @ R.T
        e += 0.5 * scene.body_mass[b] * u[b, :3] @ u[b, :3] + 0.5 * u[b, 3:] @ Iw @ u[b, 3:]
    return e


@pytest.mark.parametrize("seed", range(4))
def test_internal_impulses_conserve_momentum(orc, seed):
    rng = np.random.default_rng(seed)
    s = scenes.free_fourbar_world(rng)
    s.u[:, 3:] = 0.0  # no spin: the free velocity equals the initial one
    P = orc.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), baumgarte=0.0, eta=1e-8, rho_bil=1e-6, **TIGHT)
    out = orc.step(s, P)
    assert out["status"][0] == orc.OK
    p0, L0 = momenta(s, s.q, s.u)
    p1, L1 = momenta(s, s.q, out["u"])  # impulses act at the pre-step pose
    scale = max(np.abs(p0).max(), 1e-3)
    assert np.abs(p1 - p0).max() < 1e-10 * scale
    lscale = max(np.abs(L0).max(), 1e-3)
    assert np.abs(L1 - L0).max() < 1e-9 * lscale
    # the impulses were not trivial
    assert np.abs(out["u"] - s.u).max() > 1e-3


@pytest.mark.parametrize("seed", range(4))
def test_unbiased_step_is_a_projection(orc, seed):
    rng = np.random.default_rng(10 + seed)
    s = scenes.free_fourbar_world(rng)
    s.u[:, 3:] = 0.0
    P = orc.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), baumgarte=0.0, eta=1e-8, rho_bil=1e-6, **TIGHT)
    out = orc.step(s, P)
    S = orc.world_system(s, P, 0)
    e0, e1 = kinetic(s, s.q, s.u), kinetic(s, s.q, out["u"])
    assert e1 <= e0 * (1 + 1e-12)
    assert e1 < 0.999 * e0  # the inconsistent part of the twist was removed
    vel = S["J"] @ out["u"].reshape(-1)
    assert np.abs(vel).max() < 1e-8 * max(np.abs(s.u).max(), 1.0)


def test_rollout_keeps_the_loop_closed(orc):
    """300 steps of 1 ms: with the Baumgarte bias (beta 0.2) the largest
    constraint value (anchor gap, axis misalignment) peaks during the first
    steps, while the inconsistent initial twists are removed, stays below
    5e-5 and decays over the second half; without the bias the same rollout
    drifts several times further.  The loop is planar, so three of its
    twenty rows are redundant and the bias on them need not be consistent:
    steps may stop at the iteration cap with a small dual residual, which is
    allowed here (only non-finite results fail)."""
    rng = np.random.default_rng(3)
    s = scenes.free_fourbar_world(rng)
    final = {}
    for beta in (0.2, 0.0):
        P = orc.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), baumgarte=beta, eta=1e-8, rho_bil=1e-6, eps=1e-9,
                       max_iters=5000)
        q, u = s.q.copy(), s.u.copy()
        viol = []
        for _ in range(300):
            out = orc.step(s, P, q=q, u=u)
            assert out["status"][0] & orc.NONFINITE == 0
            q, u = out["q"], out["u"]
            viol.append(np.abs(orc.world_system(s, P, 0, q=q, u=u)["f"]).max())
        viol = np.array(viol)
        final[beta] = viol[-1]
        if beta > 0:
            assert viol.max() < 5e-5
            assert viol[150:].max() < viol[:150].max()
    assert final[0.0] > 5.0 * final[0.2]
