"""The matrix-free solve (Sec. 5.1: Delassus products through the
pre-baked Jacobian, Conjugate Residual inner solves warm-started at the
previous iterate) on the GPU, through the C ABI, against the FP64 oracle.

* The fixed figure (151 bodies, 196 joints, 45 loops: the size of the
  paper's largest system, Tab. 1; 1014 rows) runs only on this path; its
  converged step is compared with the oracle's converged solve.
* Bipeds and four-bars forced onto this path: against the oracle's own
  converged solve (unique quantities), against the oracle running the same
  Conjugate Residual budget with the GPU's restart decisions replayed
  (fixed iteration count), and against the dense GPU path.
* Batching: a figure, bipeds and four-bars in one call equal separate
  calls bit for bit; chained multi-step launches equal single steps.
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


def figure_state(n, seed):
    scene = scenes.round_to_f32(scenes.figure_batch(n, seed=1007))
    rng = np.random.default_rng(seed)
    scene = scenes.perturb_state(scene, rng, 0.05, 0.2)
    scene.u = scene.u.astype(np.float32).astype(np.float64)
    tau = np.zeros(scene.n_joints)
    act = scene.joint_actuated.astype(bool)
    tau[act] = rng.normal(0.0, 5.0, act.sum())
    return scene, tau.astype(np.float32)


def biped_state(n, seed, v_scale=0.2, w_scale=1.0):
    scene = scenes.round_to_f32(scenes.biped_batch(n, seed=1002))
    rng = np.random.default_rng(seed)
    scene = scenes.perturb_state(scene, rng, v_scale, w_scale)
    scene.u = scene.u.astype(np.float32).astype(np.float64)
    tau = np.zeros(scene.n_joints)
    act = scene.joint_actuated.astype(bool)
    tau[act] = rng.normal(0.0, 5.0, act.sum())
    return scene, tau.astype(np.float32)


def test_figure_runs_matrix_free_and_matches_oracle():
    """1014-row figures (above the dense limits, so AUTO puts them on the
    matrix-free path): u+ and J^T lambda per body within 1e-4 of the
    oracle's converged solve (its Cholesky path, to 1e-8: FP32-rounded
    loop frames leave a dual-residual floor near 3e-9)."""
    scene, tau = figure_state(4, seed=11)
    p = cfg2_params()
    m = kamx.Model(scene, params=p)
    assert [bk["rows"] for bk in m.buckets()] == [1024]
    m.close()
    g = gpu_step(scene, p, ext=tau)
    print(f"figure: iterations {g['iters'].tolist()} status {g['status'].tolist()} rows {g['rows'].tolist()}")
    assert np.all(g["status"] == 0)
    assert np.all(g["rows"] == 1014)
    rs = compare_worlds(scene, kamx.make_params(**p), g, range(4), mode="same",
                        oracle_over=dict(eps=1e-8, max_iters=20000))
    e = summary("figure, 4 worlds, matrix-free path vs oracle converged", rs)
    assert e[:, 0].max() < TOL and e[:, 1].max() < TOL


@pytest.mark.parametrize("cr_iters", [9, 25])
def test_biped_forced_matrix_free_converged(cr_iters):
    """Bipeds with probe contacts, PD and noise forced onto the matrix-free
    path: against the oracle's own converged solve (1e-12 reference), the
    unique quantities within 1e-4 and the FP64 NCP residual of the GPU
    impulses, and against the dense GPU path."""
    n = 16
    scene, tau = biped_state(n, seed=5)
    p = cfg2_params(linear_solver=kamx.SOLVER_SPARSE, cr_iters=cr_iters)
    g = gpu_step(scene, p, ext=tau)
    gd = gpu_step(scene, cfg2_params(), ext=tau)
    conv = g["status"] == 0
    print(f"biped sparse cr {cr_iters}: iterations mean {g['iters'].mean():.1f} max {g['iters'].max()} "
          f"converged {conv.mean():.3f}; dense mean {gd['iters'].mean():.1f}")
    assert conv.mean() >= 0.75
    worlds = np.nonzero(conv)[0]
    rs = compare_worlds(scene, kamx.make_params(**p), g, worlds, mode="reference")
    e = summary(f"biped, matrix-free cr {cr_iters}, {len(worlds)} converged worlds vs oracle reference", rs)
    assert e[:, 1].max() < TOL and e[:, 3].max() < TOL
    assert e[:, 4].max() < 1e-5
    both = conv & (gd["status"] == 0)
    bo = scene.body_offsets()
    for w in np.nonzero(both)[0]:
        d = np.abs(g["u"][bo[w]:bo[w + 1]] - gd["u"][bo[w]:bo[w + 1]]).max()
        s = max(np.abs(gd["u"][bo[w]:bo[w + 1]]).max(), 1e-6)
        assert d / s < 5e-4, (w, d / s)


def test_fourbar_fixed_iterations_replayed_with_the_same_budget():
    """Four-bar + sliding cube, exactly 50 ADMM iterations of 9 Conjugate
    Residual steps each: the oracle runs the same inner budget with the
    GPU's restart decisions replayed, so both paths compute the same
    iterates; u+ and J^T lambda within 1e-4 on every world."""
    scene = scenes.round_to_f32(scenes.fourbar_batch(64, seed=1001))
    p = dict(dt=1e-3, eta=1e-4, rho_bilateral=1e-6, rho_contact=1.0, fixed_iters=50, max_iters=50, log_restarts=1,
             linear_solver=kamx.SOLVER_SPARSE, cr_iters=9)
    g = gpu_step(scene, p)
    assert np.all(g["iters"] == 50)
    rs = compare_worlds(scene, kamx.make_params(**p), g, range(64), mode="replay", oracle_over=dict(cr_iters=9))
    e = summary("four-bar + box, matrix-free, 50 iterations x 9 CR steps, restarts replayed", rs)
    assert e[:, 0].max() < TOL and e[:, 1].max() < TOL


def test_drives_and_midpoint_on_the_matrix_free_path():
    """Implicit joint drives (Sec. 3, Eq. 2) with the Moreau-Jean step on
    the matrix-free path: bipeds whose chain joints are implicit PD rows,
    against the oracle's converged solve.  Twists a tenth of the Euler
    tests': at the half-step poses the redundant loop rows carry a
    second-order constraint value outside the range of J, a dual-residual
    floor growing with |u-|^2 (above 1e-6 in FP64 at sigma_w = 1 rad/s)."""
    n = 8
    scene, tau = biped_state(n, seed=9, v_scale=0.02, w_scale=0.1)
    scene = scenes.with_drives(scene, mode="implicit")
    p = cfg2_params(linear_solver=kamx.SOLVER_SPARSE, cr_iters=25, integrator=kamx.MOREAU_JEAN)
    g = gpu_step(scene, p, ext=tau)
    conv = g["status"] == 0
    print(f"drives + midpoint, matrix-free: iterations {g['iters'].tolist()}")
    assert conv.mean() >= 0.75
    # (near-static stance: the bound is the larger of 1e-4 and four times
    # the distance the oracle's own solve at the same tolerance keeps from
    # the 1e-12 reference)
    rs = compare_worlds(scene, kamx.make_params(**p), g, np.nonzero(conv)[0], mode="reference", tol_run=True)
    summary("biped with implicit drives, Moreau-Jean, matrix-free", rs)
    assert within_tolerance_bound(rs, TOL) < 1.0


def test_mixed_dense_and_matrix_free_buckets_equal_separate_calls():
    """A figure (matrix-free bucket), bipeds (224-row dense bucket) and
    four-bars (32-row dense bucket) in one model: every world's outputs
    equal those of a model holding only its own structure, bit for bit."""
    fig, tau_f = figure_state(2, seed=3)
    bp, tau_b = biped_state(3, seed=4)
    fb = scenes.round_to_f32(scenes.fourbar_batch(3, seed=1001))
    tau_fb = np.zeros(fb.n_joints, np.float32)
    mixed = scenes.concat([fig.subset([0]), bp.subset([0]), fb.subset([0]), fig.subset([1]), bp.subset([1, 2]),
                           fb.subset([1, 2])])
    tau_m = np.concatenate([tau_f[:196], tau_b[:40], tau_fb[:4], tau_f[196:], tau_b[40:], tau_fb[4:]])
    p = cfg2_params(dt=2e-3)
    # probe contacts (capacity = a world's own probe count: the figure has
    # none, so its 1016 thread rows stay within the matrix-free limit)
    gm = gpu_step(mixed, p, ext=tau_m, explicit_contacts=False, max_contacts=0)
    gf = gpu_step(fig, p, ext=tau_f, explicit_contacts=False, max_contacts=0)
    gb = gpu_step(bp, p, ext=tau_b, explicit_contacts=False, max_contacts=0)
    gfb = gpu_step(fb, p, ext=tau_fb, explicit_contacts=False, max_contacts=0)
    order = [(gf, fig, 0), (gb, bp, 0), (gfb, fb, 0), (gf, fig, 1), (gb, bp, 1), (gb, bp, 2), (gfb, fb, 1),
             (gfb, fb, 2)]
    bm, rm = mixed.body_offsets(), gm["row_offsets"]
    for k, (gs, sc, w) in enumerate(order):
        sb, rs = sc.body_offsets(), gs["row_offsets"]
        assert gm["iters"][k] == gs["iters"][w], k
        np.testing.assert_array_equal(gm["u"][bm[k]:bm[k + 1]], gs["u"][sb[w]:sb[w + 1]])
        np.testing.assert_array_equal(gm["q"][bm[k]:bm[k + 1]], gs["q"][sb[w]:sb[w + 1]])
        np.testing.assert_array_equal(gm["lam"][rm[k]:rm[k + 1]], gs["lam"][rs[w]:rs[w + 1]])


def test_chained_rollout_equals_single_steps_matrix_free():
    """Eight steps of two figures in one chained launch equal eight
    single-step calls bit for bit (positions, velocities, impulses)."""
    scene, _ = figure_state(2, seed=21)
    p = cfg2_params(torque_sigma=5.0, seed=77, log_restarts=0)
    a = kamx.Model(scene, params=p)
    a.step(8)
    b = kamx.Model(scene, params=p)
    for _ in range(8):
        b.step(1)
    torch.cuda.synchronize()
    qa, ua = a.state()
    qb, ub = b.state()
    assert torch.equal(qa, qb) and torch.equal(ua, ub)
    assert torch.equal(a.impulses(), b.impulses())
    st = a.stats()
    # (the figure's 45 loops drift under the noise: by the eighth step a
    # world may sit on a dual-residual floor and stop at the cap; what is
    # checked here is that the chained launch computes the same steps)
    print(f"figure rollout: last-step iterations {st['iters'].tolist()} status {st['status'].tolist()}")
    assert torch.all((st["status"] & ~kamx.WORLD_MAXITER) == 0)
    a.close()
    b.close()


def test_matrix_free_limits_and_unsupported_modes():
    """Worlds above the matrix-free limits are rejected at creation; the
    learned warm start and forward kinematics report EUNSUPPORTED for
    models with matrix-free worlds; forcing the dense solver on a world
    above the dense limits is rejected."""
    fig, _ = figure_state(1, seed=1)
    with pytest.raises(kamx.KamxError):
        kamx.Model(fig, params=cfg2_params(linear_solver=kamx.SOLVER_DENSE))
    with pytest.raises(kamx.KamxError):
        kamx.Model(fig, params=cfg2_params(), max_contacts=8)  # 1016 + 32 thread rows > 1024
    m = kamx.Model(fig, params=cfg2_params())
    with pytest.raises(kamx.KamxError, match="matrix-free"):
        m.features()
    with pytest.raises(kamx.KamxError):
        m.forward_kinematics(torch.zeros(fig.n_joints, device="cuda"))
    m.close()
