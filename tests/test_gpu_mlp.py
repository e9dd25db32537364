"""The warm-start network's matrix-core kernels (through the C ABI) against
the FP64 reference with the same BF16 rounding points: forward outputs,
loss, gradients and the Adam update.  The reference rounds the same
operands to BF16 and accumulates in FP64, so the differences left are the
FP32 accumulation order and rare one-unit BF16 rounding flips of hidden
activations; the bar is 2e-3 of each tensor's largest magnitude (the BF16
unit is 2^-8 = 3.9e-3; a wrong layout, transposed operand or dropped term
gives errors of order one)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mlp as M  # noqa: E402
from paper_2603_16536_amd import kamx  # noqa: E402

TOL = 2e-3


def random_net(rng, n_in, n_hidden, n_out):
    fp, op = M.pad64(n_in), M.pad64(n_out)
    W1 = np.zeros((n_hidden, fp))
    W1[:, :n_in] = rng.uniform(-1, 1, (n_hidden, n_in)) / np.sqrt(n_in)
    W3 = np.zeros((op, n_hidden))
    W3[:n_out] = rng.uniform(-1, 1, (n_out, n_hidden)) / np.sqrt(n_hidden)
    b3 = np.zeros(op)
    b3[:n_out] = rng.uniform(-0.1, 0.1, n_out)
    net = M.MLP(n_in, n_hidden, n_out, W1, rng.uniform(-0.1, 0.1, n_hidden),
                rng.uniform(-1, 1, (n_hidden, n_hidden)) / np.sqrt(n_hidden), rng.uniform(-0.1, 0.1, n_hidden),
                W3, b3,
                mu_in=np.r_[rng.normal(0, 1, n_in), np.zeros(fp - n_in)],
                s_in=np.r_[1.0 / rng.uniform(0.5, 3, n_in), np.ones(fp - n_in)],
                mu_out=np.r_[rng.normal(0, 1, n_out), np.zeros(op - n_out)],
                sigma_out=np.r_[rng.uniform(0.5, 2, n_out), np.ones(op - n_out)])
    # the device keeps FP32 parameters
    for p in net.params():
        p[...] = p.astype(np.float32)
    net.mu_in[:] = net.mu_in.astype(np.float32)
    net.mu_out[:] = net.mu_out.astype(np.float32)
    net.sigma_out[:] = net.sigma_out.astype(np.float32)
    return net


def device_net(net, max_batch):
    d = kamx.MLP(net.n_in, net.n_out, n_hidden=net.n_hidden, max_batch=max_batch, seed=1)
    assert d.n_in_pad == net.n_in_pad and d.n_out_pad == net.n_out_pad
    d.set_weights(net.packed().astype(np.float32))
    sigma_in = (1.0 / net.s_in[:net.n_in]).astype(np.float32)
    d.set_normalization(net.mu_in[:net.n_in], sigma_in, net.mu_out[:net.n_out], net.sigma_out[:net.n_out])
    # the reference uses the FP32 scale the device derives from sigma
    net.s_in[:net.n_in] = (1.0 / sigma_in.astype(np.float32)).astype(np.float32)
    return d


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


@pytest.mark.parametrize("n_in,n_hidden,n_out,batch", [(100, 128, 50, 70), (667, 256, 224, 4096)])
def test_forward_matches_reference(n_in, n_hidden, n_out, batch):
    rng = np.random.default_rng(n_in)
    net = random_net(rng, n_in, n_hidden, n_out)
    d = device_net(net, batch)
    x = rng.normal(0, 2, (batch, n_in)).astype(np.float32)
    y = d.forward(x).cpu().numpy()
    rows = np.arange(batch) if batch <= 128 else np.r_[0, 1, rng.choice(batch - 2, 62, replace=False) + 2, batch - 1]
    ref, _ = M.forward(net, x[rows].astype(np.float64), bf16=True)
    e = rel(y[rows], ref)
    print(f"\nforward {n_in}-{n_hidden}-{n_hidden}-{n_out}, batch {batch}: max error / max |y| = {e:.2e}")
    assert e < TOL
    d.close()


@pytest.mark.parametrize("n_in,n_hidden,n_out,batch,cap", [(100, 128, 50, 70, 128), (667, 256, 224, 4096, 4096),
                                                       (667, 256, 224, 1024, 4032)])
def test_gradients_loss_and_adam_match_reference(n_in, n_hidden, n_out, batch, cap):
    """Loss, the six gradients and the first Adam step.  The biped network
    at batch 4096 sums its weight gradients over the batch in several
    slices (split over the batch, slices added in order); batch 1024 under
    a capacity of 4032 (not a power of two) takes more slices than the
    capacity itself, which the workspace must hold."""
    rng = np.random.default_rng(7)
    net = random_net(rng, n_in, n_hidden, n_out)
    d = device_net(net, cap)
    x = rng.normal(0, 2, (batch, net.n_in)).astype(np.float32)
    t = (net.mu_out[:n_out] + net.sigma_out[:n_out] * rng.normal(0, 1, (batch, n_out))).astype(np.float32)
    loss_dev = torch.zeros(1, dtype=torch.float32, device="cuda")
    w0 = d.weights().cpu().numpy()
    lr = 1e-3
    d.train_step(x, t, lr, loss=loss_dev)
    g = d.gradients().cpu().numpy()
    w1 = d.weights().cpu().numpy()
    loss, grads = M.loss_and_grads(net, x.astype(np.float64), t.astype(np.float64), bf16=True)
    assert abs(loss_dev.item() - loss) <= 1e-4 * loss
    k = 0
    for name, gr in zip(["W1", "b1", "W2", "b2", "W3", "b3"], grads):
        n = gr.size
        e = rel(g[k:k + n].reshape(gr.shape), gr)
        print(f"grad {name}: max error / max |g| = {e:.2e}")
        assert e < TOL, name
        k += n
    # first Adam step: w1 = w0 - lr g / (|g| + eps) elementwise
    gref = np.concatenate([gr.ravel() for gr in grads])
    step = w0 - w1
    big = np.abs(gref) > 0.05 * np.abs(gref).max()
    expect = lr * gref / (np.abs(gref) + M.ADAM_EPS)
    assert np.abs(step[big] - expect[big]).max() < 1e-2 * lr
    assert np.abs(step).max() <= lr * 1.0001
    d.close()


def test_training_fits_a_smooth_map():
    """Adam on the device drives the loss of a smooth synthetic map down by
    more than 20x (learning check, not parity)."""
    rng = np.random.default_rng(11)
    n_in, n_out, batch = 48, 24, 512
    A = rng.normal(0, 1, (n_out, n_in)) / np.sqrt(n_in)
    x = rng.normal(0, 1, (batch, n_in)).astype(np.float32)
    t = np.tanh(x @ A.T).astype(np.float32)
    d = kamx.MLP(n_in, n_out, n_hidden=128, max_batch=batch, seed=3)
    d.set_normalization(np.zeros(n_in), np.ones(n_in), np.zeros(n_out), t.std(axis=0) + 1e-3)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    xs, ts = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    d.train_step(xs, ts, 3e-3, loss=loss)
    first = loss.item()
    for _ in range(400):
        d.train_step(xs, ts, 3e-3, loss=loss)
    print(f"\nloss {first:.3e} -> {loss.item():.3e}")
    assert loss.item() < first / 20
    d.close()


# ---- the network inside the step -------------------------------------------

from paper_2603_16536_amd import scenes  # noqa: E402

from parity_util import biped_refs, compare_world, gpu_step  # noqa: E402


def biped_model(n, params, seed=1002):
    scene = scenes.round_to_f32(scenes.biped_batch(n, seed=seed))
    return scene, kamx.Model(scene, params=params, pd=(15.0, 0.6), refs=biped_refs(scene))


BIPED = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=2000, torque_sigma=5.0,
             seed=77, contact_margin=0.02)


def slots_to_rows(pred, model, scene):
    """Host mapping of slot values to the rows of the contacts the step used."""
    raw, cnt = model.contacts()
    used = kamx.contacts_to_scene(scene, raw, cnt)
    nj = scene.joint_offsets()
    ro = model.row_offsets
    lam = np.zeros(int(ro[-1]), np.float32)
    co = used.contact_offsets()
    for w in range(scene.n_worlds):
        rc0 = 5 * (nj[w + 1] - nj[w])
        lam[ro[w]:ro[w] + rc0] = pred[w, :rc0]
        for c in range(co[w], co[w + 1]):
            k = int(used.contact_key[c])
            lam[ro[w] + rc0 + 3 * (c - co[w]):ro[w] + rc0 + 3 * (c - co[w]) + 3] = pred[w, rc0 + 3 * k:rc0 + 3 * k + 3]
    return lam, used


def test_features_and_slots_layout():
    """Features of the coming step against the state, the previous impulses
    by contact key and the torques the step then applies."""
    scene, m = biped_model(8, BIPED)
    nf, ns = m.feature_dims()
    nb, nj = 31, 40
    assert ns == 5 * nj + 3 * 8 and nf == 13 * nb + ns + nj
    m.step(2)
    x = m.features().cpu().numpy()
    prev_slots = m.impulse_slots().cpu().numpy()
    q, u = (t.cpu().numpy() for t in m.state())
    lam = m.impulses().cpu().numpy()
    raw, cnt = m.contacts()
    used = kamx.contacts_to_scene(scene, raw, cnt)
    m.step(1)
    tau = m.torques().cpu().numpy()
    co, ro = used.contact_offsets(), m.row_offsets
    for w in range(8):
        b = slice(31 * w, 31 * w + 31)
        pel = q[31 * w + scene.reset_body[w] - scene.body_offsets()[w], :3] if scene.reset_body[w] >= 0 else 0
        body = np.concatenate([q[b, :3] - pel, q[b, 3:], u[b]], axis=1).reshape(-1)
        assert np.array_equal(x[w, :13 * nb], body.astype(np.float32))
        expect = np.zeros(ns, np.float32)
        expect[:200] = lam[ro[w]:ro[w] + 200]
        for c in range(co[w], co[w + 1]):
            k = int(used.contact_key[c])
            expect[200 + 3 * k:203 + 3 * k] = lam[ro[w] + 200 + 3 * (c - co[w]):ro[w] + 203 + 3 * (c - co[w])]
        assert np.array_equal(x[w, 13 * nb:13 * nb + ns], expect)
        assert np.array_equal(prev_slots[w], expect)
        assert np.array_equal(x[w, 13 * nb + ns:], tau[40 * w:40 * w + 40])
    m.close()


def oracle_features(scene, params, w, refs):
    """Features of world w at the scene's state before its first step, on
    the oracle side: body state relative to the reset body, zero previous
    impulses, the step's joint forces."""
    from parity_util import oracle_torques
    bo = scene.body_offsets()
    b0, b1 = bo[w], bo[w + 1]
    root = scene.q[scene.reset_body[w], :3]
    body = np.concatenate([scene.q[b0:b1, :3] - root, scene.q[b0:b1, 3:], scene.u[b0:b1]], axis=1).reshape(-1)
    tau = oracle_torques(scene, params, w, step=0, pd=(15.0, 0.6), refs=refs)
    nj = len(tau)
    n_slots = 5 * nj + 3 * 8
    return np.concatenate([body, np.zeros(n_slots), tau])


def test_learned_warm_start_equals_external_and_matches_oracle():
    """Four fresh models of the same batch.  A steps warm started by its
    network; B externally with the network's device prediction placed on the
    rows (C, a cold step, reveals the contact order): A equals B bitwise.
    The oracle computes the features and the prediction itself (FP64 with
    the same BF16 rounding points, same weights); D steps externally warm
    started from that prediction and matches the oracle run from it (same
    iteration count and restart decisions).  The device prediction agrees
    with the oracle's within the network bar."""
    import torch
    import oracle
    import oracle.contacts as OC
    from parity_util import oracle_params, oracle_torques
    p = dict(BIPED, log_restarts=1)
    n = 16
    scene, A = biped_model(n, p)
    _, B = biped_model(n, p)
    _, Cm = biped_model(n, p)
    _, D = biped_model(n, p)
    refs = biped_refs(scene)
    nf, ns = A.feature_dims()
    rng = np.random.default_rng(31)
    ref_net = random_net(rng, nf, 256, ns)
    ref_net.mu_in[:] = 0.0
    ref_net.s_in[:] = 1.0
    # output scale of a trained network: centred on the oracle's converged
    # impulses of these worlds (by slot), spread a few per cent of their
    # spread across worlds
    kp0 = kamx.make_params(**p)
    csc0 = OC.probe_contacts(scene, scene.q, float(kp0.contact_margin))
    T0 = np.concatenate([oracle_torques(scene, kp0, w, pd=(15.0, 0.6), refs=refs) for w in range(n)])
    P0 = oracle_params(kp0, eps=1e-10, max_iters=20000)
    ref0 = oracle.step(csc0, P0, joint_torque=T0)
    slots = np.zeros((n, ns))
    co0 = csc0.contact_offsets()
    for w in range(n):
        r0 = int(ref0["row_offset"][w])
        slots[w, :200] = ref0["lam"][r0:r0 + 200]
        for c in range(co0[w], co0[w + 1]):
            k = int(csc0.contact_key[c])
            slots[w, 200 + 3 * k:203 + 3 * k] = ref0["lam"][r0 + 200 + 3 * (c - co0[w]):r0 + 203 + 3 * (c - co0[w])]
    ref_net.mu_out[:ns] = slots.mean(axis=0).astype(np.float32)
    ref_net.sigma_out[:ns] = (0.05 * slots.std(axis=0) + 1e-5).astype(np.float32)
    net = device_net(ref_net, n)
    # device prediction and the learned step
    pred_dev = net.forward(A.features()).cpu().numpy()
    A.attach_mlp(net)
    A.set_params(**dict(p, warmstart=kamx.WARM_LEARNED))
    A.step(1)
    Cm.step(1)
    lam_dev, _ = slots_to_rows(pred_dev, Cm, scene)
    B.set_params(**dict(p, warmstart=kamx.WARM_EXTERNAL))
    B.set_warmstart(lam_dev)
    B.step(1)
    torch.cuda.synchronize()
    qa, ua = (t.cpu().numpy() for t in A.state())
    qb, ub = (t.cpu().numpy() for t in B.state())
    assert np.array_equal(qa, qb) and np.array_equal(ua, ub)
    assert np.array_equal(A.stats()["iters"].cpu().numpy(), B.stats()["iters"].cpu().numpy())
    # oracle-side features, prediction and warm start
    kp = kamx.make_params(**dict(p, warmstart=kamx.WARM_EXTERNAL))
    kpd = kamx.make_params(**dict(p, warmstart=kamx.WARM_EXTERNAL, fixed_iters=600, max_iters=600))
    X = np.stack([oracle_features(scene, kp, w, refs) for w in range(n)])
    pred_orc, _ = M.forward(ref_net, X, bf16=True)
    e_pred = rel(pred_dev, pred_orc)
    print(f"\ndevice vs oracle prediction: {e_pred:.2e}")
    assert e_pred < TOL
    csc = OC.probe_contacts(scene, scene.q, float(kp.contact_margin))
    co = csc.contact_offsets()
    ro = A.row_offsets
    lam_orc = np.zeros(int(ro[-1]))
    for w in range(n):
        lam_orc[ro[w]:ro[w] + 200] = pred_orc[w, :200]
        for c in range(co[w], co[w + 1]):
            k = int(csc.contact_key[c])
            r = ro[w] + 200 + 3 * (c - co[w])
            lam_orc[r:r + 3] = pred_orc[w, 200 + 3 * k:203 + 3 * k]
    # D runs 600 iterations, well past convergence from any of these warm
    # starts, so the comparison holds every body (light links included) to
    # the converged answer rather than to an eps-sized band around it
    pd_ = dict(p, warmstart=kamx.WARM_EXTERNAL, fixed_iters=600, max_iters=600)
    D.set_params(**pd_)
    D.set_warmstart(lam_orc.astype(np.float32))
    D.step(1)
    torch.cuda.synchronize()
    raw, cnt = D.contacts()
    sd = {k: v.cpu().numpy() for k, v in D.stats().items()}
    g = dict(u=D.state()[1].cpu().numpy().astype(np.float64), lam=D.impulses().cpu().numpy().astype(np.float64),
             row_offsets=ro, restart_log=D.restart_log().cpu().numpy(),
             used_scene=kamx.contacts_to_scene(scene, raw, cnt),
             inputs=dict(explicit=False, step=0, ext=None, pd=(15.0, 0.6), refs=refs), **sd)
    errs = []
    for w in range(n):
        r0 = int(ro[w])
        warm = lam_orc[r0:r0 + int(sd["rows"][w])].astype(np.float32).astype(np.float64)
        errs.append(compare_world(scene, kpd, g, w, warm=warm))
    e = np.array([[d["e_u"], d["e_imp"]] for d in errs])
    print(f"learned-style warm start: iters {sd['iters'].tolist()}; max rel err u+ {e[:, 0].max():.2e} "
          f"J^T lambda {e[:, 1].max():.2e}")
    assert e[:, 1].max() < 1e-4 and e[:, 0].max() < 1e-4
    for m in (A, B, Cm, D):
        m.close()
    net.close()


def test_learned_warm_start_in_chained_launches():
    """Five steps with the network's warm start as one chained launch and as
    five single-step launches: bitwise equal states and iteration counts;
    the prediction inside the step equals the batched network's."""
    import torch
    p = dict(BIPED, log_restarts=0, warmstart=kamx.WARM_LEARNED)
    n = 16
    scene, A = biped_model(n, p)
    _, B = biped_model(n, p)
    nf, ns = A.feature_dims()
    net = kamx.MLP(nf, ns, n_hidden=256, max_batch=n, seed=12)
    net.set_normalization(np.zeros(nf), np.ones(nf) * 5.0, np.zeros(ns), np.ones(ns) * 0.01)
    A.attach_mlp(net)
    B.attach_mlp(net)
    B.set_schedule(kamx.SCHED_LPT)
    log = torch.zeros((5, n), dtype=torch.int32, device="cuda")
    A.set_iteration_log(log)
    A.step(5)
    its = []
    for _ in range(5):
        B.step(1)
        its.append(B.stats()["iters"].cpu().numpy())
    torch.cuda.synchronize()
    for x, y in zip(A.state(), B.state()):
        assert torch.equal(x, y)
    assert np.array_equal(log.cpu().numpy(), np.stack(its))
    A.close()
    B.close()
    net.close()


def test_trained_network_cuts_iterations():
    """Train the network on a short cold rollout (noise seed 2002), then run
    a rollout with a fresh noise seed cold, warm started by the previous
    step's impulses and by the network: fewer iterations with the network
    than either, and no fewer world-steps converged (status OK per step).
    The 20 chained steps are timed with events on the launch stream and
    printed; at 1024 worlds (4 per compute unit) the wall time is set by
    where the few world-steps that reach the iteration cap fall, so time
    to tolerance is compared at the benchmark's 4096 worlds, not here."""
    import torch
    from paper_2603_16536_amd import learn
    n, steps = 1024, 60
    base = dict(BIPED, log_restarts=0, seed=2002)

    def make(seed, warm):
        sc = scenes.round_to_f32(scenes.biped_batch(n, seed=1002))
        return kamx.Model(sc, params=dict(base, seed=seed, warmstart=warm), pd=(15.0, 0.6),
                          refs=np.zeros(sc.n_joints))

    net, info = learn.fit(lambda: make(2002, kamx.WARM_COLD), steps, epochs=30, batch=1024, seed=3)
    iters, status, ms = {}, {}, {}
    legs = (("cold", kamx.WARM_COLD), ("previous", kamx.WARM_PREVIOUS), ("learned", kamx.WARM_LEARNED))
    for name, warm in legs:
        times = []
        for rep in range(3):
            m = make(77, warm)
            if warm == kamx.WARM_LEARNED:
                m.attach_mlp(net)
            m.step(5)
            log = torch.zeros((20, n), dtype=torch.int32, device="cuda")
            st = torch.zeros((20, n), dtype=torch.int32, device="cuda")
            m.set_iteration_log(log, status=st)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            m.step(20)
            e1.record()
            torch.cuda.synchronize()
            if rep > 0:
                times.append(e0.elapsed_time(e1))
            iters[name] = log.cpu().numpy()
            status[name] = st.cpu().numpy()
            m.close()
        ms[name] = min(times)
    net.close()
    c, pv, l = iters["cold"].mean(), iters["previous"].mean(), iters["learned"].mean()
    ok = {k: float(np.mean(v == kamx.WORLD_OK)) for k, v in status.items()}
    print(f"\nheld-out loss {info['val_loss']:.3f}; mean iterations cold {c:.1f}, previous {pv:.1f}, learned {l:.1f}; "
          f"median {np.median(iters['cold']):.0f} -> {np.median(iters['learned']):.0f}; status OK {ok}; "
          f"20 steps: cold {ms['cold']:.1f} ms, previous {ms['previous']:.1f} ms, learned {ms['learned']:.1f} ms")
    # the rollouts are deterministic: every repetition logs the same counts
    assert l < 0.98 * c and l < pv
    assert ok["learned"] >= ok["cold"] - 1e-3


def test_box_bin_learned_warm_start():
    """Boxes in a bin with contacts generated inside the step: the learned
    warm start's contact slots are box * 8 + vertex (the contact key modulo
    512), 160 for 20 boxes, so the network is 740 -> 256 -> 256 -> 480.  A
    network fitted to cold solves of other drops steps a pile: equal, bit
    for bit, to an external warm start with its prediction put on the rows
    by slot, and each converged world against the oracle's solve from that
    warm start (the unique quantities within the distance the tolerance
    allows)."""
    from parity_util import compare_worlds, slots_to_rows, summary, within_tolerance_bound
    n = 32
    p = dict(BIPED, torque_sigma=0.0, max_iters=2000, log_restarts=0)

    def pile(seed, steps):
        sc = scenes.round_to_f32(scenes.box_bin_batch(n, seed=seed))
        m = kamx.Model(sc, params=p, max_contacts=64)
        m.contacts_box_bin(scenes.BIN_HALF, 0.01)
        m.step(steps)
        q, u = (t.cpu().numpy().astype(np.float64) for t in m.state())
        m.close()
        return sc.replace(q=q, u=u)

    # training data: cold solves along a rollout of other drops
    tr = scenes.round_to_f32(scenes.box_bin_batch(n, seed=2005))
    m = kamx.Model(tr, params=p, max_contacts=64)
    m.contacts_box_bin(scenes.BIN_HALF, 0.01)
    nf, ns = m.feature_dims()
    assert (nf, ns) == (13 * 20 + 3 * 160, 3 * 160)
    m.step(60)
    X, Y = [], []
    for _ in range(60):
        X.append(m.features().clone())
        m.step(1)
        Y.append(m.impulse_slots().clone())
    m.close()
    X, Y = torch.cat(X), torch.cat(Y)
    net = kamx.MLP(nf, ns, n_hidden=256, max_batch=X.shape[0], seed=5)
    sd_x, sd_y = X.std(0), Y.std(0)
    net.set_normalization(X.mean(0).cpu().numpy(), torch.where(sd_x > 1e-6, sd_x, torch.ones_like(sd_x)).cpu().numpy(),
                          Y.mean(0).cpu().numpy(), (sd_y + 1e-6).cpu().numpy())
    for _ in range(200):
        net.train_step(X, Y, 1e-3)
    s1 = pile(1005, 150)
    models = []
    for mode in (kamx.WARM_LEARNED, kamx.WARM_EXTERNAL, kamx.WARM_COLD):
        mm = kamx.Model(s1, params=dict(p, warmstart=mode), max_contacts=64)
        mm.contacts_box_bin(scenes.BIN_HALF, 0.01)
        models.append(mm)
    A, B, Cm = models
    pred = net.forward(A.features()).cpu().numpy()
    A.attach_mlp(net)
    A.step(1)
    Cm.step(1)
    lam_ws, used = slots_to_rows(pred, Cm, s1)
    raw, cnt = A.contacts()
    B.set_warmstart(lam_ws)
    B.step(1)
    torch.cuda.synchronize()
    for x, y in zip(A.state(), B.state()):
        assert torch.equal(x, y)
    assert torch.equal(A.impulses(), B.impulses())
    it_l, it_c = (mm.stats()["iters"].cpu().numpy() for mm in (A, Cm))
    print(f"\nbox bin, {n} piles: iterations learned mean {it_l.mean():.1f} (p50 {np.median(it_l):.0f}), "
          f"cold {it_c.mean():.1f} (p50 {np.median(it_c):.0f})")
    st = {k: v.cpu().numpy() for k, v in B.stats().items()}
    q2, u2 = (t.cpu().numpy().astype(np.float64) for t in B.state())
    g = dict(q=q2, u=u2, lam=B.impulses().cpu().numpy().astype(np.float64), row_offsets=B.row_offsets,
             used_scene=used, inputs=dict(box_bin=None, explicit=True, ext=None, step=0), **st)
    for mm in models:
        mm.close()
    worlds = np.nonzero(st["status"] == 0)[0][:8]
    assert len(worlds) >= 4
    rs = compare_worlds(used, kamx.make_params(**dict(p, warmstart=kamx.WARM_EXTERNAL)), g, worlds,
                        mode="reference", warm=lam_ws, tol_run=True)
    summary("box bin, learned warm start (as external), against the oracle from the same start", rs)
    assert within_tolerance_bound(rs, 1e-4) < 1.0
    net.close()
