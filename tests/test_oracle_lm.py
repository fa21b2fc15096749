"""Pins of the oracle's Levenberg-Marquardt variant (Sec. IV-B: Q_uu + mu I,
mu raised and the sweep retried after a failure, lowered after a success).

On a linear-quadratic problem one LM iteration accepted at alpha = 1 is the
proximal Newton step U1 = U0 - (H + mu I)^-1 g of the dense QP in the stacked
controls, H and g built here by numpy from (A, B, Q, R, Q_T); this fixes where
mu enters, the value update under a damped gain, the raise of mu to the first
power that factorises, and the floor mu0, without using the Riccati recursion.
The fall of mu from a raised value needs a Hessian that changes between
iterations: test_oracle_linesearch pins it on the point mass, whose linear
dynamics make each iteration a proximal Newton step of a dense model."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

from lq_dense import dense_qp

LQ, PM = I.SYS_LQ, I.SYS_POINT_MASS


def lm_opts(orc, **kw):
    base = dict(reg=1, eps=-np.inf, mu0=1e-6, mu_factor=10.0, mu_max=1e10)
    base.update(kw)
    return orc.Options(**base)


@pytest.mark.parametrize("mu0", [1e-3, 0.5, 20.0])
def test_lm_iteration_is_proximal_newton_step(orc, mu0):
    p = I.lq_random(4, 2, seed=9, ref=True)
    T = 12
    x0 = I.lq_x0(3, 4, seed=5)
    U0 = np.random.default_rng(1).normal(size=(3, T, 2))
    r1 = orc.solve_batch(LQ, p, x0, T, U0=U0, opts=lm_opts(orc, mu0=mu0, max_iter=1))
    r2 = orc.solve_batch(LQ, p, x0, T, U0=U0, opts=lm_opts(orc, mu0=mu0, max_iter=2))
    for b in range(3):
        H, g0, J = dense_qp(p, x0[b], T)
        Id = np.eye(H.shape[0])
        u0 = U0[b].ravel()
        u1 = u0 - np.linalg.solve(H + mu0 * Id, H @ u0 + g0)
        np.testing.assert_allclose(r1.U[b].ravel(), u1, atol=1e-10, rtol=0)
        assert abs(r1.J[b] - J(u1)) <= 1e-11 * J(u1)
        assert r1.iters[b] == 1 and r1.jtrace[b, 0] == 0
        # the accepted step lowers mu by the factor, never below mu0
        u2 = u1 - np.linalg.solve(H + mu0 * Id, H @ u1 + g0)
        np.testing.assert_allclose(r2.U[b].ravel(), u2, atol=1e-10, rtol=0)


def test_lm_converges_to_dense_optimum(orc):
    p = I.lq_random(4, 2, seed=9, ref=True)
    T = 12
    x0 = I.lq_x0(4, 4, seed=5)
    r = orc.solve_batch(LQ, p, x0, T, opts=lm_opts(orc, mu0=1e-4, max_iter=60, stop_mode=1, rtol=1e-15))
    for b in range(4):
        H, g0, J = dense_qp(p, x0[b], T)
        u = np.linalg.solve(H, -g0)
        assert abs(r.J[b] - J(u)) <= 1e-11 * abs(J(u))
        np.testing.assert_allclose(r.U[b].ravel(), u, atol=1e-7, rtol=0)


def _indefinite_lq():
    """T = 1 problem whose control Hessian H = 2 R + 2 B'Q_T B has the
    eigenvalues -3 and 5 (B = 0): unbounded below in one direction."""
    th = 0.3
    W = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    R = W @ np.diag([-1.5, 2.5]) @ W.T
    return I.lq_params(np.eye(2), np.zeros((2, 2)), np.eye(2), R, np.eye(2)), W


def test_lm_raises_mu_until_cholesky_succeeds(orc):
    p, W = _indefinite_lq()
    x0 = np.array([[1.0, -1.0]])
    U0 = np.array([[[0.7, -0.2]]])
    H, g0, J = dense_qp(p, x0[0], 1)
    assert np.allclose(np.linalg.eigvalsh(H), [-3.0, 5.0])
    # mu0 = 1e-6 times 10^k: the first mu with H + mu I positive definite is 10
    u = U0[0].ravel()
    u1 = u - np.linalg.solve(H + 10.0 * np.eye(2), H @ u + g0)
    # after the success mu falls to 1 (indefinite again) and is raised back to 10
    u2 = u1 - np.linalg.solve(H + 10.0 * np.eye(2), H @ u1 + g0)
    r1 = orc.solve_batch(LQ, p, x0, 1, U0=U0, opts=lm_opts(orc, max_iter=1))
    r2 = orc.solve_batch(LQ, p, x0, 1, U0=U0, opts=lm_opts(orc, max_iter=2))
    np.testing.assert_allclose(r1.U[0, 0], u1, atol=1e-13, rtol=0)
    np.testing.assert_allclose(r2.U[0, 0], u2, atol=1e-13, rtol=0)
    assert r2.iters[0] == 2 and r2.status[0] == orc.ST_MAX_ITER
    assert J(u2) < J(u1) < J(u)
    # the same problem under eigenvalue clipping (eq. 7): the control-cost
    # Hessian 2 R has its eigenvalue -3 raised to eps, and the step is the
    # Newton step of the clipped model
    eps = 1e-2
    Hc = W @ np.diag([eps, 5.0]) @ W.T
    uc = u - np.linalg.solve(Hc, H @ u + g0)
    rc = orc.solve_batch(LQ, p, x0, 1, U0=U0, opts=orc.Options(eps=eps, max_iter=1))
    np.testing.assert_allclose(rc.U[0, 0], uc, atol=1e-12, rtol=0)


def test_lm_gives_up_at_mu_max(orc):
    p, _ = _indefinite_lq()
    x0 = np.array([[1.0, -1.0]])
    U0 = np.array([[[0.7, -0.2]]])
    # mu may not exceed 1: every sweep fails its Cholesky, the iterate stays
    r = orc.solve_batch(LQ, p, x0, 1, U0=U0, opts=lm_opts(orc, mu_max=1.0, max_iter=5))
    assert r.status[0] == orc.ST_CHOL_FAIL and r.iters[0] == 0
    np.testing.assert_array_equal(r.U[0], U0[0])
    # a line search with no trials fails every time: mu climbs to mu_max and
    # the solve ends with a line-search failure, the iterate unchanged
    q = I.lq_random(2, 1, seed=1)
    r = orc.solve_batch(LQ, q, I.lq_x0(1, 2), 5, opts=lm_opts(orc, ls_trials=0))
    assert r.status[0] == orc.ST_LS_FAILED and r.iters[0] == 0
    assert np.all(r.U == 0)


def test_lm_solves_point_mass_to_a_stationary_point(orc):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(4, seed=3)
    T = 50
    r = orc.solve_batch(PM, p, x0, T, opts=lm_opts(orc, max_iter=200, stop_mode=1, rtol=1e-12))
    rc = orc.solve_batch(PM, p, x0, T, opts=orc.Options(max_iter=200, stop_mode=1, rtol=1e-12))
    for b in range(4):
        assert r.status[b] == orc.ST_CONVERGED
        # costs decrease monotonically along the accepted iterates
        tr = r.trace[b, :r.iters[b] + 1]
        assert np.all(np.diff(tr) < 0)
        g = orc.gradient(PM, p, x0[b], r.U[b])[3]
        assert np.max(np.abs(g)) <= 1e-4 * max(1.0, abs(r.J[b]))
        # both regularisations reach a local minimum of comparable cost
        assert abs(r.J[b] - rc.J[b]) <= 1e-3 * abs(rc.J[b])
