"""Throughput of the batched constrained-dynamics step on one MI355X.

Workload: 4096 loop-closed biped worlds (31 bodies, 40 revolute joints =
200 bilateral rows, 8 sole contact probes = up to 24 contact rows), dt =
2 ms, cold-started proximal ADMM to residual 1e-6 (cap 2000), joints driven
by PD toward the standing pose plus N(0, 5 N m) torque noise, a rollout of
--steps steps after --warmup untimed steps.  One step = one pass of the
whole hot path (bodies, rows, Delassus, factorization, PADMM, integration)
over all worlds.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VALU_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak


def biped_workload(n_worlds, seed=1002):
    from paper_2603_16536_amd import scenes
    return scenes.round_to_f32(scenes.biped_batch(n_worlds, seed=seed))


CFG2 = dict(dt=2e-3, eta=1e-4, rho_bilateral=1e-4, rho_contact=0.3, eps=1e-6, max_iters=2000,
            baumgarte=0.2, contact_margin=0.02, torque_sigma=5.0, seed=1002, reset_height=0.2,
            adapt_ratio=10.0, adapt_factor=5.0, adapt_first=100)
PD = (15.0, 0.6)   # the paper's DR Legs gains (N m / rad, N m s / rad)
WORKLOADS = {
    "biped": "biped-{n}: 31 bodies, 40 revolute joints (10 closed loops), 8 sole probes, dt 2 ms, cold-start "
             "PADMM to 1e-6 (cap 2000), PD + N(0,5 N m) torques",
    "hetero": "heterogeneous-{n}: four-bar (32 rows), biped (224 rows) and excavator (83 rows) interleaved, three "
              "concurrent size buckets, dt 2 ms, PADMM to 1e-6 (cap 200)",
    "boxbin": "box-bin-{n}: 20 boxes per world falling into a 0.3 m bin, vertex-face contacts generated every "
              "step (at most 64, 192 rows), dt 2 ms, PADMM to 1e-6 (cap 200)",
    "fourbar": "four-bar-{n}: closed four-bar (3 dynamic links, 20 rows) and a 1 kg cube sliding on the ground "
               "(4 contacts, 12 rows), dt 1 ms, exactly 50 PADMM iterations",
    "figure": "figure-{n}: 151 bodies, 196 revolute joints (45 closed loops, 980 rows), fixed to the world, dt 2 ms, "
              "explicit PD (gains capped for stability at dt) + N(0,5 N m) torques, matrix-free PADMM with {cr} "
              "Conjugate Residual iterations per iteration to 1e-6 (cap 200)",
    "biped_rl": "biped-rl-{n}: the bipeds in the paper's RL stepping setup: leg linkages driven by implicit PD rows "
                "(15 N m/rad, 0.6 N m s/rad, rotor armature and damping) + N(0,5 N m) torques, Moreau-Jean "
                "midpoint step at 250 Hz (dt 4 ms), cold-start PADMM to 1e-6 (cap 200)",
}
TRAIN_SEED = 2002  # noise seed of the rollout that feeds training (the timed rollouts use CFG2's)


def incidence_sq(scene, w=0):
    """Sum over bodies of (rows touching the body)^2 for one world with all
    of its contact probes active (an upper bound for the D assembly term)."""
    bo = scene.body_offsets()
    nb = bo[w + 1] - bo[w]
    k = np.zeros(nb)
    jo = scene.joint_offsets()
    for j in range(jo[w], jo[w + 1]):
        a, b = scene.joint_body[j]
        k[a - bo[w]] += 5
        if b >= 0:
            k[b - bo[w]] += 5
    po = scene.probe_offsets()
    for p in range(po[w], po[w + 1]):
        k[scene.probe_body[p] - bo[w]] += 3
    return float((k * k).sum())


def algorithmic_flops(rows, iters, sum_kb2):
    """Per world-step: m^3/3 (factor) + k (2 m^2 + 30 m) (iterations) +
    12 sum_b k_b^2 (Delassus assembly) + 2 m^2 (preconditioning, v_f)."""
    m = rows.astype(np.float64)
    k = iters.astype(np.float64)
    return m ** 3 / 3.0 + k * (2 * m * m + 30 * m) + 12.0 * sum_kb2 + 2 * m * m


def matrix_free_flops(rows, iters, cr_iters):
    """Per world-step of the matrix-free solve: every ADMM iteration takes
    cr_iters + 1 Delassus products through the pre-baked Jacobian (the body
    gather and the row evaluation, 12 multiply-adds each per row and side:
    48 m), about 10 m for each Conjugate Residual update and 30 m for the
    rest of the iteration; pre-baking J~ = P J M^-1/2 costs about 150 m."""
    m = rows.astype(np.float64)
    k = iters.astype(np.float64)
    return 150.0 * m + k * ((cr_iters + 1) * 48.0 * m + 10.0 * cr_iters * m + 30.0 * m)


def measured_traffic(steps_per_launch):
    """HBM bytes per step-kernel launch from the committed rocprofv3 FETCH_SIZE
    and WRITE_SIZE runs (scaled by a plain copy of known size, recorded per
    step of the batch, times the steps one launch advances), or None when the
    kernel source has changed since they were taken."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    rec = os.path.join(here, "profiles", "step_kernel_biped4096_traffic.txt")
    src = os.path.join(here, "paper_2603_16536_amd", "csrc", "kamx_step.hip")
    if not (os.path.exists(rec) and os.path.exists(src)):
        return None
    kv = dict(line.split(": ", 1) for line in open(rec).read().splitlines() if ": " in line)
    if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != kv.get("kernel_sha256_prefix"):
        return None
    return round((int(kv["fetch_bytes_per_step"]) + int(kv["write_bytes_per_step"])) * steps_per_launch)


def make_model(workload, n_worlds, warmstart, schedule, seed=None, solver="auto", cr_iters=9, extra=None,
               scene_seed=None):
    """The benchmark model of a workload: the biped batch (headline), the
    heterogeneous mix of four-bars, bipeds and excavators, boxes in a bin
    with contacts generated every step, the large fixed figure (solved
    matrix-free), or the bipeds in the paper's RL stepping setup.  solver:
    auto (dense factorization where a world fits, else matrix-free), dense
    or sparse (matrix-free for every world)."""
    from paper_2603_16536_amd import kamx, scenes

    params = dict(CFG2, warmstart=warmstart, cr_iters=cr_iters,
                  linear_solver={"auto": kamx.SOLVER_AUTO, "dense": kamx.SOLVER_DENSE,
                                 "sparse": kamx.SOLVER_SPARSE}[solver])
    if seed is not None:
        params["seed"] = seed
    params.update(extra or {})
    if workload == "biped":
        scene = biped_workload(n_worlds)
        model = kamx.Model(scene, params=params, pd=PD, refs=np.zeros(scene.n_joints))
    elif workload == "figure":
        scene = scenes.round_to_f32(scenes.figure_batch(n_worlds, seed=1007))
        # a 200-iteration budget: p99 is 25 iterations, and the few world-steps
        # that stall in FP32 would otherwise hold their workgroup for 2000
        model = kamx.Model(scene, params=dict(params, max_iters=200))
    elif workload == "hetero":
        scene = scenes.round_to_f32(scenes.heterogeneous_batch(n_worlds, seed=1003))
        # per-joint gains of each structure; a 200-iteration budget (the
        # excavator's rounded loops keep a residual floor above 1e-6)
        model = kamx.Model(scene, params=dict(params, max_iters=200))
    elif workload == "fourbar":
        scene = scenes.round_to_f32(scenes.fourbar_batch(n_worlds, seed=1001))
        # the cube's corner probes give its contacts every step
        model = kamx.Model(scene, params=dict(dt=1e-3, eta=1e-4, rho_bilateral=1e-6, rho_contact=1.0, fixed_iters=50,
                                              max_iters=50, torque_sigma=0.0, contact_margin=0.02,
                                              warmstart=warmstart, **(extra or {})),
                           max_contacts=4)
    elif workload == "biped_rl":
        scene = scenes.with_drives(scenes.round_to_f32(scenes.biped_batch(n_worlds, seed=1002, dt=4e-3, sole_probes=2)),
                                   "transmission")
        # a 200-iteration budget: at dt 4 ms most world-steps stall in FP32
        # with residuals a few times 1e-6 (the dual one at 2^-19, FP32's
        # spacing there), which a cap of 2000 does not clear either (41 %
        # converge under it); in FP64 these steps converge in under 100
        model = kamx.Model(scene, params=dict(params, dt=4e-3, integrator=kamx.MOREAU_JEAN, max_iters=200))
    elif workload == "boxbin":
        scene = scenes.round_to_f32(scenes.box_bin_batch(n_worlds, seed=1005 if scene_seed is None else scene_seed))
        model = kamx.Model(scene, params=dict(params, torque_sigma=0.0, max_iters=200), max_contacts=64)
        model.contacts_box_bin(scenes.BIN_HALF, 0.01)
    else:
        raise ValueError(workload)
    model.set_schedule(schedule)
    return scene, model


def last_step_sample(model, scene, n_sample=64, seed=0):
    """One more (untimed) step after the timed rollout, with what an FP64
    check of its solves needs: the pre-step state, the joint forces and
    contacts the step used, the impulses, the returned iterate and the
    reported residuals of a sample of worlds (every capped one first)."""
    import torch
    from paper_2603_16536_amd import kamx
    q0, u0 = (t.cpu().numpy().astype(np.float64) for t in model.state())
    it_log = model.set_iterate_log()
    model.step(1)
    torch.cuda.synchronize()
    st = {k: v.cpu().numpy() for k, v in model.stats().items()}
    raw, cnt = model.contacts()
    used = kamx.contacts_to_scene(scene.replace(q=q0, u=u0), raw, cnt)
    out = dict(scene=used, torques=model.torques().cpu().numpy().astype(np.float64),
               lam=model.impulses().cpu().numpy().astype(np.float64), row_offsets=model.row_offsets,
               iterate=it_log.cpu().numpy().astype(np.float64), **st)
    model.set_iterate_log(False)
    rng = np.random.default_rng(seed)
    capped = np.nonzero(st["status"] != 0)[0]
    rest = np.setdiff1d(np.arange(scene.n_worlds), capped)
    k = min(len(capped), n_sample // 2)
    out["sample"] = np.sort(np.r_[rng.choice(capped, k, replace=False) if k else np.zeros(0, int),
                                  rng.choice(rest, n_sample - k, replace=False)]).astype(int)
    return out


def run_gpu(n_worlds, steps, warmup, warmstart, schedule, net=None, seed=None, workload="biped", autotune=True,
            capture=False, solver="auto", cr_iters=9, extra=None):
    """Warm-up steps, then one timed call of `steps` steps (chained launches
    where the mode allows, single-step launches otherwise), bracketed by HIP
    events on the launch stream; per-step iteration and row counts come
    from the library's iteration log."""
    import torch

    scene, model = make_model(workload, n_worlds, warmstart, schedule, seed, solver, cr_iters, extra)
    if net is not None:
        model.attach_mlp(net)
    stream = torch.cuda.current_stream()
    model.step(warmup)
    torch.cuda.synchronize()
    # untimed: each size bucket keeps its fastest workgroup-size variant (the
    # state is restored, so the timed rollout continues from the warm-up)
    if autotune and any(len(b["variants"]) > 1 for b in model.buckets()):
        model.autotune(8)
    bucket_table = [f'{b["rows"]} rows x {b["worlds"]} worlds: {b["threads"]} threads' for b in model.buckets()]
    nw = scene.n_worlds
    iters = torch.zeros((steps, nw), dtype=torch.int32, device="cuda")
    rows = torch.zeros((steps, nw), dtype=torch.int32, device="cuda")
    status_log = torch.zeros((steps, nw), dtype=torch.int32, device="cuda")
    model.set_iteration_log(iters, rows, status_log)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    resets0 = model.reset_count()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    model.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    model.set_iteration_log(None)
    status = model.stats()["status"].cpu().numpy()
    check = last_step_sample(model, scene) if capture else None
    # box-bin worlds (192-row bucket) generate their contacts inside the step
    # kernel, so every workload chains under the default schedule
    chained = schedule == kamx_sched_chain()
    launches = -(-steps // 64) if chained else steps
    out = dict(
        wall_s=t1 - t0, event_ms=e0.elapsed_time(e1), launches=launches, steps_per_launch=steps / launches,
        iters=iters.cpu().numpy(), rows=rows.cpu().numpy(), status=status_log.cpu().numpy(), status_last=status,
        check=check,
        resets=model.reset_count() - resets0, buckets=model.n_buckets, bucket_table=bucket_table,
        sum_kb2=incidence_sq(scene) if workload == "biped" else 0.0,
    )
    model.close()
    return out


def mlp_throughput(net, batch=4096, reps=50):
    """Matrix-core throughput of the network's kernels on a resident batch:
    the batched forward pass and the training step (forward, backward and
    Adam), timed with HIP events on the launch stream.  Algorithmic flops:
    2 x batch x (n_in H + H H + H n_out) per forward, 8/3 of that per
    training step (three forward products; two weight-gradient and one
    activation-gradient product per layer but the first).  The training
    steps run at learning rate 0 (weights unchanged)."""
    import torch

    n_in, n_out, H = net.n_in, net.n_out, net.n_hidden
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    x = torch.randn((batch, n_in), generator=g, device="cuda")
    y = torch.randn((batch, n_out), generator=g, device="cuda")
    out = torch.empty((batch, n_out), device="cuda")
    loss = torch.zeros(1, device="cuda")
    fwd = 2.0 * batch * (n_in * H + H * H + H * n_out)
    stream = torch.cuda.current_stream()
    res = {}
    for name, fn, flops in [("forward", lambda: net.forward(x, out=out), fwd),
                            ("train_step", lambda: net.train_step(x, y, 0.0, loss=loss), fwd * 8.0 / 3.0)]:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = flops / (ms * 1e-3) / 1e12
        res[name] = {"ms": round(ms, 4), "tflops": round(tf, 3), "frac": round(tf / PEAK_BF16_MFMA_TFLOPS, 5)}
    res.update({"bound": "mfma", "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s", "batch": batch})
    return res


def solver_stats(run, world_steps):
    """Iterations and outcomes of every timed world-step (from the per-step
    iteration and status logs): a world-step converged when all three
    residuals went below 1e-6 (status OK); the rest stopped at the iteration
    cap, on a non-finite residual or a failed factorization."""
    it, st = run["iters"], run["status"]
    conv = float((st == 0).mean())
    return {"iters_mean": round(float(it.mean()), 1), "iters_p50": float(np.percentile(it, 50)),
            "iters_p99": float(np.percentile(it, 99)), "converged_fraction": round(conv, 5),
            "status_counts": {"ok": int((st == 0).sum()), "maxiter": int(((st & 1) != 0).sum()),
                              "nonfinite": int(((st & 2) != 0).sum()), "factor_fail": int(((st & 4) != 0).sum())},
            "converged_world_steps_per_s": round(world_steps * conv / run["wall_s"], 1),
            "value_counts": "every world-step, converged or stopped at the cap"}


def kamx_sched_chain():
    from paper_2603_16536_amd import kamx
    return kamx.SCHED_CHAIN


def cpu_baseline(min_seconds=12.0, n_worlds=512, max_steps=60):
    """The FP64 oracle on the host cores: the same biped workload (PD +
    noise torques, probe contacts refreshed every step, cold start to 1e-6),
    a bounded sample of worlds and steps, on every core the process may use
    and on one core."""
    import oracle

    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = min(threads, int(os.environ.get("OMP_NUM_THREADS", threads)))
    oracle.set_threads(threads)
    allc = oracle_rollout(min_seconds, n_worlds, max_steps)
    oracle.set_threads(1)
    one = oracle_rollout(min_seconds / 3.0, 32, max_steps)
    oracle.set_threads(threads)
    return dict(value=allc["rate"], unit="world-steps/s", cores=threads, kind="oracle",
                sample=f"{allc['worlds']} biped worlds x {allc['steps']} steps from the standing pose, FP64, "
                       f"mean {allc['iters']:.0f} iterations, {allc['seconds']:.1f} s",
                one_core={"value": one["rate"], "unit": "world-steps/s", "cores": 1,
                          "sample": f"{one['worlds']} worlds x {one['steps']} steps, {one['seconds']:.1f} s"})


def oracle_rollout(min_seconds, n_worlds, max_steps):
    import oracle
    from paper_2603_16536_amd import scenes

    scene = biped_workload(n_worlds)
    P = oracle.Params(dt=CFG2["dt"], eta=CFG2["eta"], rho_bil=CFG2["rho_bilateral"], rho_c=CFG2["rho_contact"],
                      eps=CFG2["eps"], max_iters=CFG2["max_iters"], baumgarte=CFG2["baumgarte"],
                      adapt_ratio=CFG2["adapt_ratio"], adapt_factor=CFG2["adapt_factor"],
                      adapt_first=CFG2["adapt_first"])
    act = np.where(scene.joint_actuated)[0]
    jo = scene.joint_offsets()
    q, u = scene.q.copy(), scene.u.copy()
    spent, done, it_sum = 0.0, 0, 0
    step = 0
    while step < max_steps and (spent < min_seconds or step == 0):
        tau = np.zeros(scene.n_joints)
        wj = scene.joint_world[act]
        u1, u2 = scenes.philox_normal_pair(CFG2["seed"], wj, step, act - jo[wj])
        noise = np.sqrt(-2.0 * np.log(u1.astype(np.float64))) * np.cos(2 * np.pi * u2.astype(np.float64))
        for i, j in enumerate(act):
            c, Ja, Jb = oracle.joint_coordinate(scene, q, j)
            a, b = scene.joint_body[j]
            rate = Ja @ u[a] + (Jb @ u[b] if b >= 0 else 0.0)
            tau[j] = PD[0] * (0.0 - c) - PD[1] * rate + CFG2["torque_sigma"] * noise[i]
        sc = contacts_from_probes(scene, q, CFG2["contact_margin"])
        t = time.perf_counter()
        out = oracle.step(sc, P, q=q, u=u, joint_torque=tau)
        spent += time.perf_counter() - t
        it_sum += int(out["iters"].sum())
        done += scene.n_worlds
        q, u = out["q"], out["u"]
        step += 1
    return dict(rate=done / spent, worlds=n_worlds, steps=step, iters=it_sum / max(done, 1), seconds=spent)


def fp64_check(chk):
    """The oracle's FP64 view of sampled GPU solves of one benchmark step:
    the natural-map NCP residual (Eq. 3) of the GPU impulses, and the three
    residuals Alg. 1 step 9 reports, recomputed at the GPU's returned
    iterate.  The system (D, v_f) is built by the oracle from the pre-step
    state, the step's joint forces and the contacts the step used."""
    import oracle

    sc = chk["scene"]
    P = oracle.Params(dt=CFG2["dt"], eta=CFG2["eta"], rho_bil=CFG2["rho_bilateral"], rho_c=CFG2["rho_contact"],
                      baumgarte=CFG2["baumgarte"], adapt_ratio=CFG2["adapt_ratio"], adapt_factor=CFG2["adapt_factor"],
                      adapt_first=CFG2["adapt_first"])
    jo = sc.joint_offsets()
    ncp_conv, ncp_all, diff = 0.0, 0.0, 0.0
    for w in chk["sample"]:
        S = oracle.world_system(sc, P, int(w), joint_torque=chk["torques"])
        m = S["J"].shape[0]
        r0 = int(chk["row_offsets"][w])
        lam = chk["lam"][r0:r0 + m]
        it = chk["iterate"][r0:r0 + m]
        D, vf, kind, mu = S["D"], S["vf"], S["kind"], S["mu"]
        p = oracle.preconditioner(D, kind)
        v = p * (D @ lam + vf)
        lt = lam / p
        r = 0.0
        i = 0
        while i < m:  # || lam~ - Pi_K(lam~ - (v + Gamma(v))) ||_inf
            if kind[i] == oracle.ROW_NORMAL:
                wv = v[i:i + 3].copy()
                wv[0] += mu[i] * np.hypot(v[i + 1], v[i + 2])
                o = oracle.project_block(2, mu[i], lt[i:i + 3] - wv)
                r = max(r, np.abs(lt[i:i + 3] - o).max())
                i += 3
            elif kind[i] == oracle.ROW_LIMIT:
                r = max(r, abs(lt[i] - max(lt[i] - v[i], 0.0)))
                i += 1
            else:
                r = max(r, abs(v[i]))
                i += 1
        ncp_all = max(ncp_all, r)
        if chk["status"][w] == 0:
            ncp_conv = max(ncp_conv, r)
            # r_p, r_d, r_c at the returned iterate with the GPU's scales
            x, y, z, pg = it[:, 0], it[:, 1], it[:, 2], it[:, 3]
            vv = pg * (D @ (pg * x)) + pg * vf
            g = np.zeros(m)
            nrm = np.nonzero(kind == oracle.ROW_NORMAL)[0]
            g[nrm] = mu[nrm] * np.hypot(vv[nrm + 1], vv[nrm + 2])
            rd = np.abs(vv + g - z).max()
            diff = max(diff, abs(rd - chk["resid"][w, 1]), abs(np.abs(x - y).max() - chk["resid"][w, 0]))
    n_conv = int(np.sum(chk["status"][chk["sample"]] == 0))
    # every sampled world-step that stopped at the cap, classified by the
    # oracle: a bilateral free velocity with a component outside the range of
    # D~_BB puts a floor under the dual residual (redundant loop rows whose
    # Baumgarte bias does not close), else the solve was merely slow
    # (the floor of |r_d|_inf lies between floor_inf = |n|_2^2 / |n|_1 and
    # |n|_2 for the component n of the bilateral free velocity outside the
    # range of D~_BB)
    floors, upper = [], []
    for w in chk["sample"]:
        if chk["status"][w] != 0:
            fr = oracle.floor_report(sc, P, int(w), joint_torque=chk["torques"])
            floors.append(fr["floor_inf"])
            upper.append(fr["floor_2"])
    floors, upper = np.array(floors), np.array(upper)
    capped = {"sampled": int(floors.size), "floor_above_eps": int(np.sum(floors > CFG2["eps"])),
              "floor_below_eps": int(np.sum(upper <= CFG2["eps"])),
              "undecided": int(np.sum((floors <= CFG2["eps"]) & (upper > CFG2["eps"]))),
              "floor_lower_bound_max": float(floors.max()) if floors.size else None,
              "floor_upper_bound_median": float(np.median(upper)) if upper.size else None,
              "floor_upper_bound_max": float(upper.max()) if upper.size else None}
    return {"ncp_residual_fp64_max_converged": float(ncp_conv), "ncp_residual_fp64_max_all": float(ncp_all),
            "capped_by_oracle_floor": capped,
            "reported_vs_fp64_residual_max_diff": float(diff), "gpu_reported_residual_max_converged":
            float(chk["resid"][chk["status"] == 0, :3].max()), "sample_worlds": len(chk["sample"]),
            "sample_converged": n_conv, "units": "preconditioned (Jacobi-scaled) impulses and velocities"}


def contacts_from_probes(scene, q, margin):
    """Explicit contacts for the oracle: sole probes below the margin."""
    from paper_2603_16536_amd.scenes import quat_to_mat
    cw, cb, cp, cg, cm, ck = [], [], [], [], [], []
    po = scene.probe_offsets()
    for w in range(scene.n_worlds):
        for k in range(po[w], po[w + 1]):
            b = scene.probe_body[k]
            pw = q[b, :3] + quat_to_mat(q[b, 3:]) @ scene.probe_point[k]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--worlds", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-previous", action="store_true", help="skip the previous-step warm-start run")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start run")
    ap.add_argument("--workload", choices=tuple(WORKLOADS), default="biped",
                    help="biped (headline), hetero (four-bar/biped/excavator mix), boxbin, fourbar, figure "
                         "or biped_rl (implicit drives, Moreau-Jean, dt 4 ms)")
    ap.add_argument("--train-steps", type=int, default=250, help="steps of the cold rollout that feeds training")
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--schedule", choices=("chain", "lpt", "index"), default="chain",
                    help="chained multi-step launches, or one launch per step ordered longest-first or by index")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep every size bucket's default workgroup size instead of the autotuner's choice")
    ap.add_argument("--solver", choices=("auto", "dense", "sparse"), default="auto",
                    help="linear solve of the x-update: dense factorization where a world fits (auto), or "
                         "matrix-free Conjugate Residual for every world (sparse)")
    ap.add_argument("--cr-iters", type=int, default=None,
                    help="Conjugate Residual iterations per ADMM iteration (default: 40 on the figure, whose 1014-row "
                         "operator with a 3e3 mass ratio needs near-exact x-updates, else 9)")
    ap.add_argument("--no-fixed-penalty", action="store_true",
                    help="skip the rollout with the fixed penalty of the paper's iteration (no adaptive penalty)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the run, copy a 256 MiB buffer once (a plain copy kernel of known traffic "
                         "for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); worlds are independent, "
              "so a multi-GPU run would shard worlds without any exchange", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_16536_amd import kamx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    kamx.lib()
    print(f"[bench] cold-start rollout: {args.worlds} worlds, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    sched = {"chain": kamx.SCHED_CHAIN, "lpt": kamx.SCHED_LPT, "index": kamx.SCHED_INDEX}[args.schedule]
    if args.cr_iters is None:
        args.cr_iters = 40 if args.workload == "figure" else 9
    if args.workload not in ("biped", "boxbin") or args.solver == "sparse":
        args.no_learned = True
    if args.workload != "biped" or args.solver == "sparse":
        args.no_cpu = True
    sparse = args.workload == "figure" or args.solver == "sparse"
    cold = run_gpu(args.worlds, args.steps, args.warmup, kamx.WARM_COLD, sched, workload=args.workload,
                   autotune=not args.no_autotune, capture=args.workload == "biped" and not args.no_cpu and not sparse,
                   solver=args.solver, cr_iters=args.cr_iters)
    value = args.worlds * args.steps / cold["wall_s"]
    it = cold["iters"]
    conv = float((cold["status"] == 0).mean())
    if sparse:
        flops_total = float(matrix_free_flops(cold["rows"], it, args.cr_iters).sum())
    else:
        flops_total = float(algorithmic_flops(cold["rows"], it, cold["sum_kb2"]).sum())
    avg_launch_s = cold["event_ms"] / 1e3 / cold["launches"]
    achieved = flops_total / cold["launches"] / avg_launch_s / 1e12
    result = {
        "metric": "world-steps/s at 4096 worlds, residual<=1e-6: plain vs learned warm-start",
        "value": round(value, 1),
        "unit": "world-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * cold["wall_s"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].format(n=args.worlds, cr=args.cr_iters),
                   "linear_solve": (f"matrix-free, {args.cr_iters} Conjugate Residual iterations per ADMM iteration"
                                    if sparse else "dense factorization once per step"),
                   "worlds": args.worlds, "rows_per_world_max": int(cold["rows"].max()),
                   "warm_start": "cold (plain ADMM)",
                   "dispatch": {"chain": "each world kept on its workgroup for up to 64 steps per launch",
                                "lpt": "one launch per step, longest previous solve first",
                                "index": "one launch per step, world index order"}[args.schedule],
                   "buckets": cold["bucket_table"]},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 5),
                     "traffic": (measured_traffic(cold["steps_per_launch"])
                                 if args.workload == "biped" and args.worlds == 4096 and not sparse else None),
                     "kernel": ("sparse_step_kernel" if sparse else
                                "step_kernel<224,512>" if args.workload == "biped" else "all step kernels"),
                     "avg_launch_ms": round(1e3 * avg_launch_s, 4), "steps_per_launch": cold["steps_per_launch"]},
        "solver": solver_stats(cold, args.worlds * args.steps),
    }
    result["config"]["penalty"] = ("per-row rho (bilateral 1e-4, limit and contact 0.3), the limit and contact rows' "
                                   "share adapted by residual balancing (ratio 10, factor 5, at iterations 100 * 2^j; "
                                   "not in the paper)")
    result["solver"]["resets"] = int(cold["resets"])
    if not args.no_fixed_penalty:
        print("[bench] fixed-penalty rollout (the paper's iteration as printed)", file=sys.stderr, flush=True)
        fx = run_gpu(args.worlds, args.steps, args.warmup, kamx.WARM_COLD, sched, workload=args.workload,
                     autotune=not args.no_autotune, solver=args.solver, cr_iters=args.cr_iters,
                     extra=dict(adapt_ratio=0.0))
        result["fixed_penalty"] = {
            "value": round(args.worlds * args.steps / fx["wall_s"], 1),
            "ms_per_step": round(1e3 * fx["wall_s"] / args.steps, 4),
            **solver_stats(fx, args.worlds * args.steps)}
    if not args.no_previous:
        print("[bench] previous-step warm-start rollout", file=sys.stderr, flush=True)
        prev = run_gpu(args.worlds, args.steps, args.warmup, kamx.WARM_PREVIOUS, sched, workload=args.workload,
                       autotune=not args.no_autotune, solver=args.solver, cr_iters=args.cr_iters)
        result["warm_previous"] = {
            "value": round(args.worlds * args.steps / prev["wall_s"], 1),
            "ms_per_step": round(1e3 * prev["wall_s"] / args.steps, 4),
            **solver_stats(prev, args.worlds * args.steps)}
    if not args.no_learned:
        from paper_2603_16536_amd import learn
        print(f"[bench] learned warm start: {args.train_steps}-step cold rollout for data (noise seed "
              f"{TRAIN_SEED}), {args.epochs} epochs", file=sys.stderr, flush=True)
        t0 = time.perf_counter()

        def factory():
            # the same structure under another noise seed (biped) or other
            # drops of the boxes (box bin)
            _, m = make_model(args.workload, args.worlds, kamx.WARM_COLD, sched, seed=TRAIN_SEED,
                              scene_seed=TRAIN_SEED + 3)
            return m

        net, info = learn.fit(factory, args.train_steps, epochs=args.epochs, batch=min(4096, args.worlds), lr=1e-3,
                              seed=1004, log=lambda msg: print(f"[bench]   {msg}", file=sys.stderr, flush=True),
                              capacity=args.worlds)
        t_train = time.perf_counter() - t0
        print("[bench] learned warm-start rollout", file=sys.stderr, flush=True)
        lrn = run_gpu(args.worlds, args.steps, args.warmup, kamx.WARM_LEARNED, sched, net=net, workload=args.workload,
                      autotune=not args.no_autotune)
        result["learned"] = {
            "value": round(args.worlds * args.steps / lrn["wall_s"], 1),
            "ms_per_step": round(1e3 * lrn["wall_s"] / args.steps, 4),
            "speedup_vs_plain": round((args.worlds * args.steps / lrn["wall_s"]) / value, 4),
            **solver_stats(lrn, args.worlds * args.steps),
            "network": f"{net.n_in} -> {net.n_hidden} -> {net.n_hidden} -> {net.n_out} (GELU), BF16 matrix-core "
                       "kernels, FP32 accumulation",
            "training": {"samples": info["samples"], "held_out": info["held_out"], "epochs": args.epochs,
                         "final_train_loss": round(info["train_loss"][-1], 5), "val_loss": round(info["val_loss"], 5),
                         "data_and_training_s": round(t_train, 2), "noise_seed": TRAIN_SEED},
            "network_kernels": mlp_throughput(net, batch=min(4096, args.worlds))}
        net.close()
    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline()
        if cold["check"] is not None:
            print("[bench] FP64 check of sampled GPU solves", file=sys.stderr, flush=True)
            result["solver"]["fp64_check"] = fp64_check(cold["check"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
