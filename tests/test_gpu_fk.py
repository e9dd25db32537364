"""Forward kinematics for resets on the GPU (through the C ABI; Sec. 6.3)
against the oracle's Gauss-Newton and the closed forms it is pinned to.

The joint frames reach the library in FP32, and rounded frames of a planar
loop are not exactly parallel: the loop's redundant constraints then have
no exact common solution, and |F|_inf stops at a floor of about 1e-7 (the
oracle's FP64 Gauss-Newton on the same rounded frames stops there too).
The tolerance is set just above it."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2603_16536_amd import kamx, scenes  # noqa: E402


def rot(q):
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


FK_TOL = 3e-7


def gpu_fk(scene, targets, max_iters=50, tol=FK_TOL):
    m = kamx.Model(scene)
    it, res = m.forward_kinematics(targets, max_iters=max_iters, tol=tol)
    q, u = (t.cpu().numpy().astype(np.float64) for t in m.state())
    it, res = it.cpu().numpy(), res.cpu().numpy()
    m.close()
    return q, u, it, res


def test_biped_random_targets_match_oracle():
    """4096 bipeds (the benchmark's batch), random targets on the ten chain
    joints: the GPU's poses equal the oracle's within FP32 rounding of the
    poses, every constraint holds at the returned FP32 poses, the targets
    are reached and the pelvis is untouched."""
    n = 4096
    scene = scenes.round_to_f32(scenes.biped_batch(n, seed=1002))
    rng = np.random.default_rng(3)
    targets = np.full(scene.n_joints, np.nan)
    act = scene.joint_actuated.astype(bool)
    targets[act] = rng.uniform(-0.3, 0.3, act.sum()).astype(np.float32)
    scene.u[:] = rng.normal(0.0, 0.1, scene.u.shape)
    q, u, it, res = gpu_fk(scene, targets)
    print(f"\niterations max {it.max()} mean {it.mean():.2f}; |F|_inf (FP64 poses) max {res.max():.2e}")
    assert np.all(res <= FK_TOL) and np.all(it <= 20)
    assert np.all(u == 0.0)
    bo = scene.body_offsets()
    pel = bo[:-1] + scene.reset_body - bo[:-1]
    assert np.array_equal(q[pel], scene.q[pel])
    worlds = rng.choice(n, size=32, replace=False)
    sub = scene.subset(worlds)
    sel = np.concatenate([np.arange(scene.joint_offsets()[w], scene.joint_offsets()[w + 1]) for w in worlds])
    qo, ito, reso = oracle.forward_kinematics(sub, targets[sel], tol=1e-12, max_iters=30)
    print(f"oracle |F|_inf on the same FP32 frames: {reso.min():.1e} .. {reso.max():.1e}")
    qg = np.concatenate([q[bo[w]:bo[w + 1]] for w in worlds])
    err_p = np.abs(qg[:, :3] - qo[:, :3]).max()
    err_r = max(np.abs(rot(a[3:]) - rot(b[3:])).max() for a, b in zip(qg, qo))
    P = oracle.Params(dt=2e-3)
    sg = sub.replace(q=qg)
    f_max = max(np.abs(oracle.world_system(sg, P, k)["f"][:200]).max() for k in range(len(worlds)))
    c_err = max(abs(oracle.joint_coordinate(sg, qg, j)[0] - targets[sel][j]) for j in np.nonzero(~np.isnan(targets[sel]))[0])
    print(f"vs oracle: positions {err_p:.2e} m, rotations {err_r:.2e}; constraint residual at FP32 poses {f_max:.2e}; "
          f"target error {c_err:.2e}")
    assert err_p < 2e-6 and err_r < 2e-6
    assert f_max < 2e-6 and c_err < 2e-6


def test_fourbar_crank_targets_follow_loop_closure():
    rng = np.random.default_rng(5)
    worlds = [scenes.fourbar_world(rng, with_box=False) for _ in range(16)]
    metas = [w.meta for w in worlds]
    scene = scenes.round_to_f32(scenes.concat(worlds))
    deltas = rng.uniform(-0.15, 0.15, 16)
    targets = np.full(scene.n_joints, np.nan)
    targets[scene.joint_offsets()[:-1]] = deltas.astype(np.float32)
    q, u, it, res = gpu_fk(scene, targets)
    assert np.all(res <= FK_TOL)
    O = np.array([0.0, 0.0, 0.6])
    bo = scene.body_offsets()
    worst = 0.0
    for w, geo in enumerate(metas):
        th2 = geo["th2"] - float(np.float32(deltas[w]))
        P = np.array([geo["a"] * math.cos(th2), geo["a"] * math.sin(th2)])
        e = geo["D"] - P
        dist = np.linalg.norm(e)
        x = (dist * dist + geo["b"] ** 2 - geo["c"] ** 2) / (2 * dist)
        h = math.sqrt(geo["b"] ** 2 - x * x)
        ex = e / dist
        Q = P + x * ex + h * np.array([-ex[1], ex[0]])
        r = bo[w] + 2
        rocker_end = q[r, :3] + rot(q[r, 3:]) @ np.array([0.5 * geo["c"], 0.0, 0.0])
        worst = max(worst, np.abs(rocker_end - (O + np.array([Q[0], 0.0, Q[1]]))).max())
    print(f"\nrocker pin vs the loop-closure closed form: {worst:.2e} m (inputs rounded to FP32)")
    assert worst < 5e-6


def test_too_many_target_rows_leave_the_world_unchanged():
    """A biped with every one of its 40 joints targeted needs 240 rows (more
    than a world's 224): the world keeps its poses and reports NaN; the
    other world (ten targets) is solved."""
    scene = scenes.round_to_f32(scenes.biped_batch(2, seed=1002))
    targets = np.full(scene.n_joints, np.nan)
    targets[:40] = 0.0
    act = scene.joint_actuated.astype(bool)
    targets[40:][act[40:]] = 0.1
    q, u, it, res = gpu_fk(scene, targets)
    assert np.isnan(res[0]) and it[0] == 0 and np.isfinite(res[1]) and res[1] <= FK_TOL
    assert np.array_equal(q[:31], scene.q[:31])


def test_reset_from_fk_then_rollout():
    """Randomised resets (Sec. 6.3): FK to random chain-joint targets, the
    result uploaded as the reset state, then a 50-step PD rollout.  Away from
    the assembled pose the FP32-rounded loop axes are no longer exactly
    parallel, the three redundant rows of each loop become nearly (not
    exactly) dependent and some solves run to the cap (the oracle in FP64
    behaves the same on these states); the rollout must stay finite with
    most steps converged."""
    n = 256
    scene = scenes.round_to_f32(scenes.biped_batch(n, seed=1002))
    rng = np.random.default_rng(9)
    targets = np.full(scene.n_joints, np.nan)
    act = scene.joint_actuated.astype(bool)
    targets[act] = rng.uniform(-0.1, 0.1, act.sum())
    m = kamx.Model(scene, params=dict(torque_sigma=1.0, seed=3))
    it, res = m.forward_kinematics(targets)
    q, u = m.state()
    m.upload_state(q, u, as_reset_state=True)
    log = torch.zeros((50, n), dtype=torch.int32, device="cuda")
    m.set_iteration_log(log)
    m.step(50)
    st = m.stats()
    torch.cuda.synchronize()
    iters = log.cpu().numpy()
    print(f"\nFK residual max {res.max().item():.1e}; rollout iterations mean {iters.mean():.1f}, "
          f"capped {np.mean(iters >= 2000):.4f}")
    assert res.max().item() <= FK_TOL
    assert np.mean(iters >= 2000) < 0.25
    assert torch.isfinite(q).all() and np.all(st["status"].cpu().numpy() & kamx.WORLD_NONFINITE == 0)
    m.close()
