"""Pins of the oracle's adaptive penalty on limit and contact rows.

Not in the paper (its penalty rho is fixed through a solve, Alg. 1): residual
balancing after Boyd, Parikh, Chu, Peleato and Eckstein (2011, Sec. 3.4.1),
applied to the unilateral rows' share of the per-row penalty.  At the
checkpoint iterations first * 2^j the rule compares the dual and primal
residuals of that iteration: r_d > tau r_p divides the unilateral penalty by
f, r_p > tau r_d multiplies it by f; a change refactors
D~ + diag(eta + rho) and restarts the acceleration at the current iterate.

* the rule on two decoupled unit-diagonal rows, worked out by hand (the
  reduction of the restart tests with the penalty changes added), with the
  limit row separating and with it pressed;
* switched off, or with a ratio that never fires, the solve is the plain one
  bit for bit;
* the converged answer does not depend on it: frictionless contact against
  the enumerated LCP solution, with changes forced early;
* what it is for: biped world-steps that the fixed penalty leaves at the
  iteration cap converge.
"""
import math

import numpy as np
import pytest

from paper_2603_16536_amd import scenes


def is_checkpoint(k, first):
    return k >= first and k % first == 0 and ((k // first) & (k // first - 1)) == 0


def two_row_adaptive(n_iters, eta, rho_a, rho_b, gamma, tau, f, first):
    """The two-row problem of the restart tests (D~ = I; row a free with
    v~_a = -1, row b a separating limit row with v~_b = 1/2; cold start)
    with the penalty rule.  While y_b stays 0 (checked):
    x_a,k = (1 + eta x_a,k-1 + rho_a y^_a,k-1) / (1 + eta + rho_a),
    x_b,k = (-1/2 + eta x_b,k-1 + z^_b,k-1) / (1 + eta + rho_b),
    z_b,k = z^_b,k-1 - rho_b x_b,k; r_p = |x_b|,
    r_d = max(|x_a - 1|, |x_b + 1/2 - z_b|); the restart test on
    c = rho_a (y_a - y^_a)^2 + (z_b - z^_b)^2 / rho_b.  At a checkpoint, after
    the extrapolation: rho_b / f if r_d > tau r_p, rho_b f if r_p > tau r_d
    (row a is bilateral and keeps rho_a), then a = 1, c_prev = inf,
    y^ = y, z^ = z.  Returns per iteration (log byte, x_a, x_b, z_b, rho_b)
    with the restart in bit 0 and the change in bits 1-2 (1 lowered, 2
    raised)."""
    xa = yha = ypa = 0.0
    xb = zhb = zpb = 0.0
    a, c_prev = 1.0, math.inf
    out = []
    for k in range(1, n_iters + 1):
        xa_n = (1.0 + eta * xa + rho_a * yha) / (1.0 + eta + rho_a)
        xb_n = (-0.5 + eta * xb + zhb) / (1.0 + eta + rho_b)
        assert xb_n - zhb / rho_b <= 0.0  # y_b stays 0
        zb_n = zhb - rho_b * xb_n
        c = rho_a * (xa_n - yha) ** 2 + (zb_n - zhb) ** 2 / rho_b
        restart = not c < gamma * c_prev
        if not restart:
            a_n = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a * a))
            beta = (a - 1.0) / a_n
            yha = xa_n + beta * (xa_n - ypa)
            zhb = zb_n + beta * (zb_n - zpb)
            a, c_prev = a_n, c
        else:
            yha, zhb = ypa, zpb
            a, c_prev = 1.0, c_prev / gamma
        xa, ypa, xb, zpb = xa_n, xa_n, xb_n, zb_n
        rp, rd = abs(xb_n), max(abs(xa_n - 1.0), abs(xb_n + 0.5 - zb_n))
        d = 0
        if is_checkpoint(k, first):
            if rd > tau * rp:
                d, rho_b = 1, rho_b / f
            elif rp > tau * rd:
                d, rho_b = 2, rho_b * f
            if d:
                a, c_prev = 1.0, math.inf
                yha, zhb = xa_n, zb_n
        out.append((int(restart) | d << 1, xa_n, xb_n, zb_n, rho_b))
    return out


def two_row_pressed(n_iters, eta, rho_a, rho_b, gamma, tau, f, first):
    """Row a as above, row b a limit row pressed by v~_b = -1/2, so that
    y_b = x_b - z^_b / rho_b stays positive (checked) and the projection never
    acts: z stays 0 on both rows, y = x, r_p = 0 exactly, and
    x_a,k = (1 + eta x_a,k-1 + rho_a y^_a,k-1) / (1 + eta + rho_a),
    x_b,k = (1/2 + eta x_b,k-1 + rho_b y^_b,k-1) / (1 + eta + rho_b);
    r_d = max(|x_a - 1|, |x_b - 1/2|); c = rho_a (y_a - y^_a)^2 +
    rho_b (y_b - y^_b)^2.  At a checkpoint r_d > tau r_p = 0 divides rho_b
    by f and restarts the acceleration (while r_d > 0).
    Returns per iteration (log byte, x_a, x_b, rho_b)."""
    xa = yha = ypa = 0.0
    xb = yhb = ypb = 0.0
    a, c_prev = 1.0, math.inf
    out = []
    for k in range(1, n_iters + 1):
        xa_n = (1.0 + eta * xa + rho_a * yha) / (1.0 + eta + rho_a)
        xb_n = (0.5 + eta * xb + rho_b * yhb) / (1.0 + eta + rho_b)
        assert xb_n > 0.0  # the limit row stays pressed
        c = rho_a * (xa_n - yha) ** 2 + rho_b * (xb_n - yhb) ** 2
        restart = not c < gamma * c_prev
        if not restart:
            a_n = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * a * a))
            beta = (a - 1.0) / a_n
            yha = xa_n + beta * (xa_n - ypa)
            yhb = xb_n + beta * (xb_n - ypb)
            a, c_prev = a_n, c
        else:
            yha, yhb = ypa, ypb
            a, c_prev = 1.0, c_prev / gamma
        xa, ypa, xb, ypb = xa_n, xa_n, xb_n, xb_n
        rd = max(abs(xa_n - 1.0), abs(xb_n - 0.5))
        d = 0
        if is_checkpoint(k, first) and rd > 0.0:
            d, rho_b = 1, rho_b / f
            a, c_prev = 1.0, math.inf
            yha, yhb = xa_n, xb_n
        out.append((int(restart) | d << 1, xa_n, xb_n, rho_b))
    return out


def test_rule_on_two_decoupled_rows(orc):
    eta, ra, rb, gamma, tau, f, first = 0.1, 0.5, 1.0, 0.999, 1.5, 2.0, 2
    ref = two_row_adaptive(40, eta, ra, rb, gamma, tau, f, first)
    # hand outcome: lowered at 8, raised at 16, lowered at 32 (checkpoints
    # 2 and 4 leave the penalty alone)
    assert [(k + 1, r[0] >> 1) for k, r in enumerate(ref) if r[0] >> 1] == [(8, 1), (16, 2), (32, 1)]
    D = np.diag([4.0, 0.25])
    vf = np.array([-2.0, 0.25])  # Jacobi scales (1/2, 2): D~ = I, v~ = (-1, 1/2)
    kind = np.array([orc.ROW_BILATERAL, orc.ROW_LIMIT], np.int32)
    mu = np.zeros(2)
    P = orc.Params(eta=eta, rho_bil=ra, rho_c=rb, restart_factor=gamma, eps=0.0, adapt_ratio=tau, adapt_factor=f,
                   adapt_first=first)
    for k in (3, 7, 8, 9, 12, 16, 17, 25, 32, 33, 40):
        o = orc.solve_ncp(D, vf, kind, mu, P.replace(fixed_iters=k), log_iters=k)
        assert list(o["restart_log"]) == [r[0] for r in ref[:k]], k
        _, xa, xb, zb, _ = ref[k - 1]
        assert abs(o["lam_tilde"][0] - xa) < 1e-13
        assert o["lam_tilde"][1] == 0.0
        assert abs(o["resid"][0] - abs(xb)) < 1e-13
        assert abs(o["resid"][1] - max(abs(xa - 1.0), abs(xb + 0.5 - zb))) < 1e-13
    # pressed limit row (v~_b = -1/2): lowered at every checkpoint 2, 4, 8, 16
    # (by iteration 32 both rows reach their fixed point exactly, r_d = 0, so
    # the comparison stops at 30, clear of that boundary)
    ref = two_row_pressed(30, eta, ra, rb, gamma, tau, f, first)
    assert [(k + 1, r[0] >> 1) for k, r in enumerate(ref) if r[0] >> 1] == [(2, 1), (4, 1), (8, 1), (16, 1)]
    vf = np.array([-2.0, -0.25])  # Jacobi scales (1/2, 2): D~ = I, v~ = (-1, -1/2)
    for k in (1, 2, 3, 5, 8, 9, 16, 17, 24, 29, 30):
        o = orc.solve_ncp(D, vf, kind, mu, P.replace(fixed_iters=k), log_iters=k)
        assert list(o["restart_log"]) == [r[0] for r in ref[:k]], k
        _, xa, xb, _ = ref[k - 1]
        assert abs(o["lam_tilde"][0] - xa) < 1e-13 and abs(o["lam_tilde"][1] - xb) < 1e-13
        assert o["resid"][0] == 0.0
        assert abs(o["resid"][1] - max(abs(xa - 1.0), abs(xb - 0.5))) < 1e-13


def biped_states(orc, n_worlds, steps, seed=1002):
    """World-steps of a short cold-started biped rollout (PD toward the
    standing pose plus N(0, 5 N m) noise, probe contacts below 2 cm), as
    (scene with the pre-step state and its contacts, joint forces)."""
    import oracle.contacts as OC
    scene = scenes.round_to_f32(scenes.biped_batch(n_worlds, seed=seed))
    P = orc.Params(dt=2e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-6, max_iters=2000)
    act = np.where(scene.joint_actuated)[0]
    jo, bo = scene.joint_offsets(), scene.body_offsets()
    rng = np.random.default_rng(seed)
    q, u = scene.q.copy(), scene.u.copy()
    out = []
    for step in range(steps):
        tau = np.zeros(scene.n_joints)
        for j in act:
            c, Ja, Jb = orc.joint_coordinate(scene, q, j)
            a, b = scene.joint_body[j]
            rate = Ja @ u[a] + (Jb @ u[b] if b >= 0 else 0.0)
            tau[j] = -15.0 * c - 0.6 * rate + 5.0 * rng.normal()
        sc = OC.probe_contacts(scene.replace(q=q, u=u), q, 0.02)
        res = orc.step(sc, P, q=q, u=u, joint_torque=tau)
        out.append((sc.replace(q=q.copy(), u=u.copy()), tau, res))
        q, u = res["q"], res["u"]
    return P, out


def test_off_or_never_firing_is_the_plain_solve(orc):
    P, steps = biped_states(orc, 8, 3)
    for sc, tau, plain in steps:
        for over in (dict(adapt_ratio=0.0), dict(adapt_ratio=1e300, adapt_first=1)):
            o = orc.step(sc, P.replace(**over), joint_torque=tau)
            assert np.array_equal(o["u"], plain["u"]) and np.array_equal(o["lam"], plain["lam"])
            assert np.array_equal(o["iters"], plain["iters"])


def test_frictionless_contact_answer_unchanged(orc):
    """Penalty changes forced from the second iteration on, on a box resting
    on three points of its lower face under gravity with a small random
    twist: the converged normal impulses are the unique solution of the
    enumerated LCP, the changes did happen, and most scenes have a pressed
    contact."""
    n_changed = n_pressed = 0
    for seed in range(6):
        rng = np.random.default_rng(seed)
        s = scenes.box_point_contacts(rng, n_points=3, mu=0.0, gap_scale=0.0, v_scale=0.02)
        P = orc.Params(dt=1e-3, baumgarte=0.2, rho_c=1.0, eps=1e-13, max_iters=200000, adapt_ratio=1.5,
                       adapt_factor=3.0, adapt_first=2)
        out = orc.step(s, P, log_iters=64)
        assert out["status"][0] == orc.OK, seed
        n_changed += int(np.any(out["restart_log"][0] >> 1))
        S = orc.world_system(s, P, 0)
        D, vf = S["D"], S["vf"]
        nrm = np.arange(0, 9, 3)
        Dn, vn = D[np.ix_(nrm, nrm)], vf[nrm]
        sols = []
        for mask in range(8):
            act = [k for k in range(3) if mask >> k & 1]
            lam = np.zeros(3)
            if act:
                lam[act] = np.linalg.solve(Dn[np.ix_(act, act)], -vn[act])
            v = Dn @ lam + vn
            if np.all(lam >= -1e-12) and np.all(v >= -1e-12):
                sols.append(lam)
        assert len(sols) == 1, seed
        assert np.abs(out["lam"][nrm] - sols[0]).max() < 1e-9 * max(1.0, np.abs(sols[0]).max()), seed
        n_pressed += int(np.any(sols[0] > 0.0))
    assert n_changed == 6 and n_pressed >= 4, (n_changed, n_pressed)


def test_capped_biped_world_steps_converge(orc):
    """Biped world-steps that stop at the 2000-iteration cap with the fixed
    penalty (1-2 % of a rollout; in about half of them r_p falls to 1e-12
    while r_d stays at 1e-6 for 20000 iterations) converge with the rule at
    tau = 10 (the usual residual-balancing ratio), f = 5 from iteration 100;
    the others are no slower."""
    orc.set_threads(8)
    P, steps = biped_states(orc, 48, 24)
    PA = P.replace(adapt_ratio=10.0, adapt_factor=5.0, adapt_first=100)
    capped, slower, n = 0, 0, 0
    conv = 0
    for sc, tau, plain in steps:
        o = orc.step(sc, PA, joint_torque=tau)
        n += sc.n_worlds
        cap = plain["status"] != orc.OK
        capped += int(cap.sum())
        conv += int(np.sum(o["status"][cap] == orc.OK))
        slower += int(np.sum((o["iters"] > 1.05 * plain["iters"] + 5) & ~cap))
    print(f"\n{n} world-steps: {capped} capped with the fixed penalty, {conv} of them converge with the rule; "
          f"{slower} converged ones slower by more than 5 %")
    assert capped >= 5
    assert conv >= 0.7 * capped
    assert slower <= 0.01 * n
