"""Invariants of the GPU step that hold at any batch size (Sec. 3:
constraint impulses are internal forces; the velocity update of Eq. 2 is a
projection), on 4096 closed four-bar loops floating free of the world
without gravity, with random twists: linear and angular momentum of every
world are unchanged by the step, kinetic energy does not increase, the
constraint velocities vanish to the solver tolerance, and over a rollout
with the Baumgarte bias the loops stay closed."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2603_16536_amd import kamx, scenes  # noqa: E402

from test_oracle_invariants import kinetic, momenta  # noqa: E402

N = 4096


def params(**over):
    p = dict(dt=1e-3, gravity=(0.0, 0.0, 0.0), eta=1e-6, rho_bilateral=1e-6, rho_contact=1.0, eps=1e-6,
             max_iters=2000, baumgarte=0.0, log_restarts=0)
    p.update(over)
    return p


def test_step_conserves_momentum_and_does_not_add_energy():
    scene = scenes.round_to_f32(scenes.free_fourbar_batch(N, seed=1006))
    scene.u[:, 3:] = 0.0  # no spin: no gyroscopic term in the free velocity
    m = kamx.Model(scene, params=params())
    m.step(1)
    torch.cuda.synchronize()
    u = m.state()[1].cpu().numpy().astype(np.float64)
    st = m.stats()["status"].cpu().numpy()
    m.close()
    assert np.mean(st == 0) > 0.99
    bo = scene.body_offsets()
    e_p, e_l, ratio = [], [], []
    for w in range(N):
        sub = scene.subset([w])
        b0, b1 = bo[w], bo[w + 1]
        p0, L0 = momenta(sub, sub.q, sub.u)
        p1, L1 = momenta(sub, sub.q, u[b0:b1])
        e_p.append(np.abs(p1 - p0).max() / max(np.abs(p0).max(), 1e-3))
        e_l.append(np.abs(L1 - L0).max() / max(np.abs(L0).max(), 1e-3))
        ratio.append(kinetic(sub, sub.q, u[b0:b1]) / kinetic(sub, sub.q, sub.u))
    e_p, e_l, ratio = np.array(e_p), np.array(e_l), np.array(ratio)
    print(f"\n{N} free loops: linear momentum rel. change max {e_p.max():.2e}, angular {e_l.max():.2e}, "
          f"kinetic energy ratio max {ratio.max():.6f} mean {ratio.mean():.3f}", flush=True)
    assert e_p.max() < 1e-5 and e_l.max() < 1e-5
    assert ratio.max() <= 1.0 + 1e-5


def test_constraint_velocities_vanish_after_the_step():
    """Without the bias the solve drives the preconditioned constraint
    velocities p_i (J u+)_i below eps = 1e-6 (the dual residual on free
    rows); u+ is stored in FP32, which adds about 1e-7."""
    scene = scenes.round_to_f32(scenes.free_fourbar_batch(64, seed=7))
    m = kamx.Model(scene, params=params())
    m.step(1)
    torch.cuda.synchronize()
    u = m.state()[1].cpu().numpy().astype(np.float64)
    st = m.stats()["status"].cpu().numpy()
    m.close()
    P = oracle.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), baumgarte=0.0)
    bo = scene.body_offsets()
    worst = 0.0
    for w in range(64):
        if st[w] != 0:
            continue
        sub = scene.subset([w])
        S = oracle.world_system(sub, P, 0)
        p = 1.0 / np.sqrt(np.diag(S["D"]))
        v = p * (S["J"] @ u[bo[w]:bo[w + 1]].reshape(-1))
        worst = max(worst, np.abs(v).max())
    print(f"\nconverged worlds {np.mean(st == 0):.3f}; max |p (J u+)| = {worst:.2e}", flush=True)
    assert np.mean(st == 0) > 0.95 and worst < 5e-6


def test_rollout_keeps_the_loops_closed():
    """300 chained steps on 4096 loops with and without the Baumgarte bias:
    on 64 sampled worlds the largest constraint value after the rollout is
    below 5e-4 with the bias, and the bias cuts it at least threefold in
    the median world."""
    scene = scenes.round_to_f32(scenes.free_fourbar_batch(N, seed=1006))
    final = {}
    for beta in (0.2, 0.0):
        m = kamx.Model(scene, params=params(baumgarte=beta, max_iters=400))
        m.step(300)
        torch.cuda.synchronize()
        final[beta] = m.state()[0].cpu().numpy().astype(np.float64)
        m.close()
    P = oracle.Params(dt=1e-3, gravity=(0.0, 0.0, 0.0), baumgarte=0.2)
    rng = np.random.default_rng(0)
    bo = scene.body_offsets()
    viol = {0.2: [], 0.0: []}
    for w in rng.choice(N, 64, replace=False):
        sub = scene.subset([int(w)])
        for beta, q in final.items():
            viol[beta].append(np.abs(oracle.world_system(sub, P, 0, q=q[bo[w]:bo[w + 1]])["f"]).max())
    vb, v0 = np.array(viol[0.2]), np.array(viol[0.0])
    print(f"\nafter 300 steps: max constraint value {vb.max():.2e} with the bias, {v0.max():.2e} without; "
          f"median ratio {np.median(vb / v0):.3f}", flush=True)
    assert np.all(np.isfinite(final[0.2])) and vb.max() < 5e-4
    assert np.median(vb / v0) < 1.0 / 3.0
