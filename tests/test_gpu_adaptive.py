"""The adaptive penalty on limit and contact rows on the GPU (through the C
ABI), against the oracle's rule (the oracle is pinned in
tests/test_oracle_adaptive.py; the rule is not in the paper, whose penalty
is fixed through a solve).

* 4096 perturbed bipeds in one call, with and without the rule: worlds that
  stop at the cap with the fixed penalty converge with it, and the others
  take no more iterations;
* worlds whose penalty changed: the oracle replays the GPU's iteration
  count, restart decisions and penalty changes (log bits 0 and 1-2), so
  both compute the same iterates: u+ and J^T lambda within 1e-4; against the
  oracle's own converged solve with the rule, the unique quantities within
  the distance the tolerance allows;
* the matrix-free path changes the penalty without refactoring and gives
  the dense path's answers.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16536_amd import kamx, scenes  # noqa: E402

from parity_util import compare_worlds, gpu_step, summary, within_tolerance_bound  # noqa: E402

TOL = 1e-4


def cfg2_params(**over):
    p = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=2000, log_restarts=1)
    p.update(over)
    return p


def biped_state(n_worlds, seed):
    scene = scenes.round_to_f32(scenes.biped_batch(n_worlds, seed=1002))
    rng = np.random.default_rng(seed)
    scene = scenes.perturb_state(scene, rng, 0.2, 1.0)
    scene.u = scene.u.astype(np.float32).astype(np.float64)
    tau = np.zeros(scene.n_joints)
    act = scene.joint_actuated.astype(bool)
    tau[act] = rng.normal(0.0, 5.0, act.sum())
    return scene, tau.astype(np.float32)


def test_defaults_switch_the_rule_on():
    p = kamx.default_params()
    assert p.adapt_ratio == 10.0 and p.adapt_factor == 5.0 and p.adapt_first == 100
    with pytest.raises(kamx.KamxError):
        kamx.Model(scenes.round_to_f32(scenes.fourbar_batch(1, seed=1001)), params=dict(adapt_factor=0.5))


def test_capped_worlds_converge_and_replay_matches_the_oracle():
    scene, tau = biped_state(4096, seed=7)
    g = gpu_step(scene, cfg2_params(), ext=tau)
    g0 = gpu_step(scene, cfg2_params(adapt_ratio=0.0), ext=tau)
    changed = ((g["restart_log"] >> 1) & 3).any(axis=1)
    cap0 = g0["status"] != kamx.WORLD_OK
    print(f"\nfixed penalty: {cap0.sum()} of 4096 capped, iterations mean {g0['iters'].mean():.1f}; "
          f"adaptive: {np.sum(g['status'] != 0)} capped, iterations mean {g['iters'].mean():.1f}; "
          f"penalty changed in {changed.sum()} worlds", flush=True)
    assert np.sum(g["status"] != 0) <= 0.75 * cap0.sum()
    assert g["iters"].mean() < g0["iters"].mean()
    # a world whose penalty never changed ran the fixed-penalty iterations
    same = ~changed
    assert np.array_equal(g["iters"][same], g0["iters"][same])
    assert np.array_equal(g["u"][np.repeat(same, scene.n_bodies // scene.n_worlds)],
                          g0["u"][np.repeat(same, scene.n_bodies // scene.n_worlds)])
    worlds = np.nonzero(changed)[0][:16]
    assert len(worlds) >= 4
    params = kamx.make_params(**cfg2_params())
    rs = compare_worlds(scene, params, g, worlds, mode="replay")
    e = summary(f"{len(worlds)} worlds whose penalty changed, oracle replaying the GPU's decisions", rs)
    assert e[:, 0].max() < TOL and e[:, 1].max() < TOL
    conv = [w for w in worlds if g["status"][w] == 0]
    rs = compare_worlds(scene, params, g, conv, mode="reference", tol_run=True)
    summary(f"{len(conv)} of them converged, against the oracle's own solve with the rule", rs)
    assert within_tolerance_bound(rs, TOL) < 1.0


def test_matrix_free_path_changes_the_penalty_without_refactoring():
    scene, tau = biped_state(64, seed=11)
    ps = cfg2_params(linear_solver=kamx.SOLVER_SPARSE, cr_iters=25)
    g = gpu_step(scene, ps, ext=tau)
    changed = ((g["restart_log"] >> 1) & 3).any(axis=1)
    print(f"\nmatrix-free: penalty changed in {changed.sum()} of 64 worlds; converged {np.mean(g['status'] == 0):.3f}")
    gd = gpu_step(scene, cfg2_params(), ext=tau)
    both = (g["status"] == 0) & (gd["status"] == 0)
    assert both.mean() > 0.9
    bo = scene.body_offsets()
    for w in np.nonzero(both)[0]:
        d = np.abs(g["u"][bo[w]:bo[w + 1]] - gd["u"][bo[w]:bo[w + 1]]).max()
        s = max(np.abs(gd["u"][bo[w]:bo[w + 1]]).max(), 1e-6)
        assert d / s < 5e-4, (w, d / s)
    worlds = np.nonzero(changed & (g["status"] == 0))[0][:6]
    if len(worlds):
        rs = compare_worlds(scene, kamx.make_params(**ps), g, worlds, mode="replay", oracle_over=dict(cr_iters=25))
        e = summary("matrix-free worlds whose penalty changed, replayed with the same CR budget", rs)
        assert e[:, 0].max() < TOL and e[:, 1].max() < TOL
