"""Pins of the oracle's iterative inner solve (Sec. 5.1: Conjugate Residual
on the Delassus operator with a fixed budget, warm-started at the previous
ADMM iterate):

* Conjugate Residual minimises the residual norm over growing Krylov
  spaces: its residual norm never grows, and on an n x n SPD system it
  reaches the direct solution (in n iterations in exact arithmetic; a few
  n in floating point, where the directions lose conjugacy);
* inside Alg. 1 with the paper's budget of 9 iterations, the ADMM iteration
  reaches the same fixed point as with the exact (Cholesky) solve: on
  redundant loops, frictionless and frictional contacts and the biped, the
  unique quantities (u+, J^T lambda) agree and the NCP residual (Eq. 3) at
  the returned impulses is as small.
"""
import numpy as np
import pytest

from paper_2603_16536_amd import scenes


@pytest.mark.parametrize("n", [5, 24, 60])
def test_cr_reaches_the_direct_solution_and_never_increases_the_residual(orc, n):
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.logspace(0, 3, n)) @ Q.T
    b = rng.normal(size=n)
    x_ref = np.linalg.solve(A, b)
    assert np.abs(orc.cr_solve(A, b, 4 * n) - x_ref).max() < 1e-8 * np.abs(x_ref).max()
    res = [np.linalg.norm(b - A @ orc.cr_solve(A, b, k)) for k in range(n + 1)]
    assert all(r1 <= r0 * (1 + 1e-12) for r0, r1 in zip(res, res[1:]))
    # warm start: from the exact solution there is nothing left to do
    assert np.abs(orc.cr_solve(A, b, 3, x0=x_ref) - x_ref).max() < 1e-12 * np.abs(x_ref).max()


def worlds():
    rng = np.random.default_rng(7)
    out = [scenes.fourbar_world(rng, with_box=False) for _ in range(2)]
    out += [scenes.box_point_contacts(rng, n_points=3, mu=0.0, gap_scale=1e-3, v_scale=0.3)]
    out += [scenes.box_point_contacts(rng, n_points=4, mu=0.6, gap_scale=1e-3, v_scale=0.3)]
    b = scenes.biped_batch(2, seed=1002)
    b = scenes.perturb_state(b, rng, 0.2, 1.0)
    out += [b.subset([0]), b.subset([1])]
    return scenes.concat(out, dt=1e-3)


def test_padmm_with_cr_reaches_the_cholesky_fixed_point(orc):
    s = worlds()
    P = orc.Params(dt=1e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-12, max_iters=200000)
    dense = orc.step(s, P)
    cr = orc.step(s, P.replace(cr_iters=9))
    assert np.all(dense["status"] == 0) and np.all(cr["status"] == 0)
    print("\niterations dense", dense["iters"], "CR(9)", cr["iters"])
    assert np.abs(cr["u"] - dense["u"]).max() < 1e-8 * max(1.0, np.abs(dense["u"]).max())
    ro = dense["row_offset"]
    for w in range(s.n_worlds):
        S = orc.world_system(s, P, w)
        imp_d = S["J"].T @ dense["lam"][ro[w]:ro[w + 1]]
        imp_c = S["J"].T @ cr["lam"][ro[w]:ro[w + 1]]
        assert np.abs(imp_c - imp_d).max() < 1e-8 * max(1e-6, np.abs(imp_d).max()), w
    assert cr["resid"][:, 3].max() < 1e-10


def test_cr_budget_changes_iterations_not_the_answer(orc):
    """A budget of 1, 3 and 30 CR iterations: the ADMM iteration count moves,
    the converged velocities do not."""
    s = worlds()
    P = orc.Params(dt=1e-3, eta=1e-4, rho_bil=1e-4, rho_c=0.3, eps=1e-11, max_iters=400000)
    ref = orc.step(s, P)
    for n in (1, 3, 30):
        o = orc.step(s, P.replace(cr_iters=n))
        assert np.all(o["status"] == 0), n
        assert np.abs(o["u"] - ref["u"]).max() < 1e-7 * max(1.0, np.abs(ref["u"]).max()), n
