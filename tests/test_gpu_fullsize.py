"""Parity at the full batch sizes of the heterogeneous and contact-heavy
configurations, in the launch configuration of the benchmark (one model,
every size bucket, contacts generated on the device): sampled worlds of the
single GPU step against the oracle replay of the same iterations and
restart decisions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16536_amd import kamx, scenes  # noqa: E402

from parity_util import compare_world, compare_worlds, summary  # noqa: E402

TOL = 1e-4


def test_heterogeneous_8192_worlds_sampled():
    """8192 worlds (four-bar, biped and excavator interleaved), three size
    buckets with the autotuner's workgroup sizes, PD + noise actuation and
    probe contacts generated on the device, a 200-iteration budget.  Four-bars
    and bipeds: net impulses per body within 1e-4 and u+ within 5e-4 (the
    3-30 g transmission links); excavators: net impulses and the
    momentum-weighted u+ error within 1e-4."""
    scene = scenes.round_to_f32(scenes.heterogeneous_batch(8192, seed=1003))
    p = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=200, torque_sigma=5.0,
             seed=1003, log_restarts=1)
    m = kamx.Model(scene, params=p)
    m.autotune(2)
    m.step(1)
    torch.cuda.synchronize()
    q, u = (t.cpu().numpy().astype(np.float64) for t in m.state())
    st = {k: v.cpu().numpy() for k, v in m.stats().items()}
    g = dict(q=q, u=u, lam=m.impulses().cpu().numpy().astype(np.float64), row_offsets=m.row_offsets,
             restart_log=m.restart_log().cpu().numpy(), **st)
    raw, cnt = m.contacts()
    g["used_scene"] = kamx.contacts_to_scene(scene, raw, cnt)
    g["inputs"] = dict(ext=None, explicit=False, step=0, pd=None, refs=None)
    print("\nbuckets:", m.buckets(), flush=True)
    m.close()
    kp = kamx.make_params(**p)
    rng = np.random.default_rng(3)
    for kind, name in enumerate(["four-bar", "biped", "excavator"]):
        ws = np.sort(rng.choice(np.arange(kind, 8192, 3), size=2, replace=False))
        errs = [compare_world(scene, kp, g, int(w)) for w in ws]
        e_u = max(x["e_u"] for x in errs)
        e_imp = max(x["e_imp"] for x in errs)
        e_mom = max(x["e_mom"] for x in errs)
        print(f"{name} worlds {ws.tolist()}, iters {g['iters'][ws].tolist()}: u+ {e_u:.2e} J^T lambda {e_imp:.2e} "
              f"momentum-weighted u+ {e_mom:.2e}", flush=True)
        assert e_imp < TOL and e_mom < TOL
        if name != "excavator":
            assert e_u < 5 * TOL


def test_box_bin_16384_worlds_sampled():
    """16384 worlds of twelve resting boxes in a bin (contacts generated on
    the device, at most 64 per world), one step: contact keys exact, u+ and
    net impulses per body within 1e-4 on sampled worlds."""
    scene = scenes.round_to_f32(scenes.box_bin_resting_batch(16384, seed=1005))
    p = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=2000, log_restarts=1)
    margin = 0.004
    m = kamx.Model(scene, params=p, max_contacts=64)
    m.contacts_box_bin(scenes.BIN_HALF, margin)
    m.step(1)
    torch.cuda.synchronize()
    q, u = (t.cpu().numpy().astype(np.float64) for t in m.state())
    st = {k: v.cpu().numpy() for k, v in m.stats().items()}
    g = dict(q=q, u=u, lam=m.impulses().cpu().numpy().astype(np.float64), row_offsets=m.row_offsets,
             restart_log=m.restart_log().cpu().numpy(), **st)
    raw, cnt = m.contacts()
    g["used_scene"] = kamx.contacts_to_scene(scene, raw, cnt)
    g["inputs"] = dict(box_bin=(scenes.BIN_HALF[0], scenes.BIN_HALF[1], margin, 64), ext=None, step=0)
    m.close()
    counts = cnt.cpu().numpy()
    print(f"\ncontacts per world: min {counts.min()} mean {counts.mean():.1f} max {counts.max()}", flush=True)
    assert counts.min() > 0 and counts.max() <= 64
    kp = kamx.make_params(**p)
    ws = np.sort(np.random.default_rng(5).choice(16384, size=4, replace=False))
    errs = [compare_world(scene, kp, g, int(w)) for w in ws]
    e = np.array([[x["e_u"], x["e_imp"], x["r_ncp"]] for x in errs])
    print(f"\nbox bin 16384 worlds, sample {ws.tolist()}, iters {g['iters'][ws].tolist()}: u+ {e[:, 0].max():.2e} "
          f"J^T lambda {e[:, 1].max():.2e} FP64 r_ncp {e[:, 2].max():.2e}; converged "
          f"{np.mean(g['status'] == 0):.4f}", flush=True)
    assert e[:, 0].max() < TOL and e[:, 1].max() < TOL


def test_figure_4096_worlds_matrix_free_sampled():
    """4096 fixed figures (1014 rows each, matrix-free) in the benchmark's
    launch configuration: 40 Conjugate Residual iterations per x-update, a
    200-iteration budget, explicit PD toward the assembled pose plus noise
    torques, from perturbed twists.  At least 99 % converge; on sampled
    converged worlds, u+ and the net impulse per body within 1e-4 of the
    oracle's own solve (exact x-updates by Cholesky, to 1e-8)."""
    scene = scenes.round_to_f32(scenes.figure_batch(4096, seed=1007))
    rng = np.random.default_rng(13)
    scene = scenes.perturb_state(scene, rng, 0.05, 0.2)
    scene.u = scene.u.astype(np.float32).astype(np.float64)
    p = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=200, torque_sigma=5.0,
             seed=1007, cr_iters=40, log_restarts=1)
    m = kamx.Model(scene, params=p)
    assert [bk["rows"] for bk in m.buckets()] == [1024]
    m.step(1)
    torch.cuda.synchronize()
    q, u = (t.cpu().numpy().astype(np.float64) for t in m.state())
    st = {k: v.cpu().numpy() for k, v in m.stats().items()}
    g = dict(q=q, u=u, lam=m.impulses().cpu().numpy().astype(np.float64), row_offsets=m.row_offsets,
             restart_log=m.restart_log().cpu().numpy(), **st)
    raw, cnt = m.contacts()
    g["used_scene"] = kamx.contacts_to_scene(scene, raw, cnt)
    g["inputs"] = dict(ext=None, explicit=False, step=0, pd=None, refs=None)
    m.close()
    conv = st["status"] == 0
    print(f"\nfigure 4096: iterations mean {st['iters'].mean():.1f} max {st['iters'].max()}, converged {conv.mean():.4f}",
          flush=True)
    assert conv.mean() >= 0.99
    ws = np.sort(rng.choice(np.nonzero(conv)[0], size=6, replace=False))
    rs = compare_worlds(scene, kamx.make_params(**p), g, ws, mode="same",
                        oracle_over=dict(cr_iters=0, eps=1e-8, max_iters=20000))
    e = summary(f"figure 4096, worlds {ws.tolist()}, matrix-free (40 CR iterations) vs oracle converged", rs)
    assert e[:, 0].max() < TOL and e[:, 1].max() < TOL
