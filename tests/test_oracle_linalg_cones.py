"""Pins of the oracle's dense factorization and of the cone projections
(Sec. 3 cones, Alg. 1 step 6).  The projection onto the Coulomb cone K_mu is
checked through Moreau's decomposition, which characterises it uniquely:
w = Pi_K(w) + Pi_Ko(w) with Pi_K(w) in K, w - Pi_K(w) in the polar cone
-K* (K* = {mu |v_t| <= v_n}), and the two parts orthogonal."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st


def test_cholesky_reconstructs_random_spd(orc):
    rng = np.random.default_rng(0)
    for n in [1, 2, 5, 17, 32, 64]:
        G = rng.normal(size=(n, n))
        A = G @ G.T + 1e-3 * np.eye(n)
        L, rc = orc.cholesky(A)
        assert rc == 0
        assert np.allclose(np.triu(L, 1), 0.0)
        assert np.abs(L @ L.T - A).max() <= 1e-12 * np.abs(A).max()


def test_cholesky_reports_first_non_positive_pivot(orc):
    A = np.diag([4.0, 1.0, -1.0, 2.0])
    _, rc = orc.cholesky(A)
    assert rc == -3  # -1 - (index of the failing column)
    B = np.array([[1.0, 2.0], [2.0, 1.0]])  # indefinite
    _, rc = orc.cholesky(B)
    assert rc == -2


floats = st.floats(min_value=-10.0, max_value=10.0, allow_nan=False, allow_infinity=False)


@settings(max_examples=300, deadline=None)
@given(w=st.tuples(floats, floats, floats), mu=st.floats(min_value=0.0, max_value=2.0))
def test_coulomb_projection_moreau(orc, w, mu):
    w = np.array(w)
    o = orc.project_block(2, mu, w)
    r = w - o
    tol = 1e-12 * (1.0 + np.abs(w).max())
    # o in K_mu
    assert np.hypot(o[1], o[2]) <= mu * o[0] + tol
    # w - o in the polar cone: -(w - o) in K* = {mu |v_t| <= v_n}
    assert mu * np.hypot(r[1], r[2]) <= -r[0] + tol
    # orthogonality
    assert abs(o @ r) <= tol * (1.0 + np.abs(w).max())
    # idempotence
    assert np.abs(orc.project_block(2, mu, o) - o).max() <= tol


def test_coulomb_projection_special_cases(orc):
    mu = 0.5
    inside = np.array([1.0, 0.2, 0.3])
    assert np.array_equal(orc.project_block(2, mu, inside), inside)
    polar = np.array([-1.0, 0.1, 0.0])  # mu |t| <= -n
    assert np.array_equal(orc.project_block(2, mu, polar), np.zeros(3))
    # tie-break at zero tangential part: stays on the normal axis
    assert np.array_equal(orc.project_block(2, mu, np.array([-0.0, 0.0, 0.0])), np.zeros(3))
    # mu = 0: projection on the normal ray
    o = orc.project_block(2, 0.0, np.array([0.7, 0.4, -0.2]))
    assert np.allclose(o, [0.7, 0.0, 0.0])


def test_limit_and_free_projections(orc):
    assert orc.project_block(1, 0.0, np.array([-0.3]))[0] == 0.0
    assert orc.project_block(1, 0.0, np.array([0.3]))[0] == 0.3
    assert orc.project_block(0, 0.0, np.array([-0.3]))[0] == -0.3
