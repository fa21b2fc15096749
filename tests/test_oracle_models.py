"""Pins of the oracle's system models (dynamics, costs, derivatives) against
mathematics that does not go through the oracle's own formulas: exact linear
maps, finite differences of function values, energy conservation and the
kinetic-energy definition of the mass matrix."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

PM, P3, QUAD = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_QUAD_SYNTH


def fd_jac(fun, z, h=1e-6):
    """Central-difference Jacobian of fun at z (4th-order stencil)."""
    z = np.asarray(z, float)
    f0 = np.asarray(fun(z))
    J = np.zeros((f0.size, z.size))
    for j in range(z.size):
        e = np.zeros_like(z)
        e[j] = h
        J[:, j] = (-fun(z + 2 * e) + 8 * fun(z + e) - 8 * fun(z - e) + fun(z - 2 * e)) / (12 * h)
    return J


SYSTEMS = [
    (PM, I.point_mass_params(0), lambda rng: np.r_[rng.uniform(-2, 2, 2), rng.uniform(-1, 1, 2)], 2),
    (P3, I.planar3_params(0), lambda rng: np.r_[rng.uniform(-3, 3, 3), rng.uniform(-1, 1, 3)], 3),
    (QUAD, I.quad_params(0), lambda rng: np.r_[rng.uniform(-1, 1, 19), rng.uniform(-0.5, 0.5, 18)], 12),
]


def test_point_mass_dynamics_is_the_exact_semi_implicit_double_integrator(orc):
    p = I.point_mass_params(3)
    dt = p[0]
    A = np.array([[1, 0, dt, 0], [0, 1, 0, dt], [0, 0, 1, 0], [0, 0, 0, 1]], float)
    B = np.array([[dt * dt, 0], [0, dt * dt], [dt, 0], [0, dt]], float)
    rng = np.random.default_rng(0)
    for _ in range(10):
        x, u = rng.normal(size=4), rng.normal(size=2)
        np.testing.assert_allclose(orc.dyn(PM, p, x, u), A @ x + B @ u, rtol=0, atol=1e-15)
        Aj, Bj = orc.dyn_jac(PM, p, x, u)
        np.testing.assert_allclose(Aj, A, atol=1e-15)
        np.testing.assert_allclose(Bj, B, atol=1e-15)


@pytest.mark.parametrize("kind,params,xs,m", SYSTEMS, ids=["pm", "arm", "quad"])
def test_dynamics_jacobians_match_finite_differences(orc, kind, params, xs, m):
    rng = np.random.default_rng(1)
    n, mm = orc.dims(kind, params)
    assert mm == m
    for _ in range(3):
        x, u = xs(rng), rng.normal(size=m)
        A, B = orc.dyn_jac(kind, params, x, u)
        Afd = fd_jac(lambda z: orc.dyn(kind, params, z, u), x)
        Bfd = fd_jac(lambda z: orc.dyn(kind, params, x, z), u)
        np.testing.assert_allclose(A, Afd, rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(B, Bfd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("kind,params,xs,m", SYSTEMS, ids=["pm", "arm", "quad"])
def test_cost_derivatives_match_finite_differences(orc, kind, params, xs, m):
    rng = np.random.default_rng(2)
    n, _ = orc.dims(kind, params)
    for _ in range(3):
        x, u = xs(rng), rng.normal(size=m)
        lx, lu, lxx, luu, lux = orc.cost_derivs(kind, params, x, u)
        z = np.r_[x, u]
        f = lambda zz: np.array([orc.cost(kind, params, zz[:n], zz[n:])])
        g = fd_jac(f, z)[0]
        np.testing.assert_allclose(lx, g[:n], rtol=1e-7, atol=1e-8)
        np.testing.assert_allclose(lu, g[n:], rtol=1e-7, atol=1e-8)
        # Hessian against second differences of the cost value itself
        H = fd_jac(lambda zz: fd_jac(f, zz, h=1e-4)[0], z, h=1e-4)
        np.testing.assert_allclose(lxx, H[:n, :n], rtol=1e-4, atol=1e-5)
        np.testing.assert_allclose(luu, H[n:, n:], rtol=1e-4, atol=1e-5)
        assert np.all(lux == 0.0)  # no state-control cross terms in these costs
        lTx, lTxx = orc.term_derivs(kind, params, x)
        ft = lambda zz: np.array([orc.term(kind, params, zz)])
        np.testing.assert_allclose(lTx, fd_jac(ft, x)[0], rtol=1e-7, atol=1e-8)
        HT = fd_jac(lambda zz: fd_jac(ft, zz, h=1e-4)[0], x, h=1e-4)
        np.testing.assert_allclose(lTxx, HT, rtol=1e-4, atol=1e-5)


def test_point_mass_cost_special_values(orc):
    p = I.point_mass_params(0)
    g = p[5:7]
    # at the goal with zero velocity the terminal cost vanishes
    assert orc.term(PM, p, np.r_[g, 0.0, 0.0]) == 0.0
    # at an obstacle centre its Gaussian contributes exactly w_obs
    q = p.copy()
    q[[7, 8]] = [0.3, -0.2]
    q[[10, 11, 13, 14]] = [1e3, 1e3, 1e3, 1e3]  # other obstacles far away
    l = orc.cost(PM, q, np.array([0.3, -0.2, 5.0, 5.0]), np.array([1.0, -2.0]))
    expect = q[1] * 5.0 + q[2] * ((0.3 - g[0]) ** 2 + (-0.2 - g[1]) ** 2) + q[4] * 1.0
    assert abs(l - expect) < 1e-14 * max(1.0, expect)


def _arm_energy(p, x):
    """Kinetic energy of the three uniform rods, from centre-of-mass velocities
    obtained by differentiating the link geometry (not from a mass matrix)."""
    m, L = p[1:4], p[4:7]
    q, qd = x[:3], x[3:]

    def coms(qq):
        phi = np.cumsum(qq)
        out, base = [], np.zeros(2)
        for i in range(3):
            d = np.array([np.cos(phi[i]), np.sin(phi[i])])
            out.append(base + 0.5 * L[i] * d)
            base = base + L[i] * d
        return np.concatenate(out)

    h = 1e-6
    v = (coms(q + h * qd) - coms(q - h * qd)) / (2 * h)
    w = np.cumsum(qd)
    E = 0.0
    for i in range(3):
        E += 0.5 * m[i] * (v[2 * i] ** 2 + v[2 * i + 1] ** 2) + 0.5 * (m[i] * L[i] ** 2 / 12) * w[i] ** 2
    return E


def test_arm_mass_matrix_is_the_kinetic_energy_metric(orc):
    p = I.planar3_params(1)
    rng = np.random.default_rng(3)
    for _ in range(5):
        x = np.r_[rng.uniform(-3, 3, 3), rng.uniform(-2, 2, 3)]
        M = orc.p3_mass(p, x[:3])
        assert np.allclose(M, M.T, atol=1e-15)
        assert np.linalg.eigvalsh(M).min() > 0
        assert abs(0.5 * x[3:] @ M @ x[3:] - _arm_energy(p, x)) < 1e-8


def test_arm_end_effector_geometry(orc):
    p = I.planar3_params(2)
    L = p[4:7]
    np.testing.assert_allclose(orc.p3_ee(p, np.zeros(3)), [L.sum(), 0.0], atol=1e-15)
    np.testing.assert_allclose(orc.p3_ee(p, np.array([np.pi / 2, 0, 0])), [0.0, L.sum()], atol=1e-14)
    np.testing.assert_allclose(orc.p3_ee(p, np.array([0.0, np.pi, 0])), [L[0] - L[1] - L[2], 0.0],
                               atol=1e-14)


def test_arm_conserves_energy_without_torque_and_balances_power(orc):
    # With tau = 0 the continuous-time arm conserves kinetic energy; a wrong
    # sign or index in the velocity-product term would make it drift.
    p = I.planar3_params(0).copy()
    p[0] = 1e-4
    x = np.array([0.3, -1.1, 0.7, 1.5, -2.0, 2.5])
    E0 = _arm_energy(p, x)
    for _ in range(2000):
        x = orc.dyn(P3, p, x, np.zeros(3))
    assert abs(_arm_energy(p, x) - E0) < 1e-3 * E0
    # with torque, energy change equals the work tau^T dq
    x = np.array([0.3, -1.1, 0.7, 0.5, -0.4, 0.6])
    tau = np.array([0.2, -0.1, 0.05])
    E0, work = _arm_energy(p, x), 0.0
    for _ in range(2000):
        xn = orc.dyn(P3, p, x, tau)
        work += tau @ (xn[:3] - x[:3])
        x = xn
    assert abs((_arm_energy(p, x) - E0) - work) < 2e-3 * abs(work)


def test_quad_dynamics_properties(orc):
    p = I.quad_params(0)
    dt = p[0]
    # rest at qb = 0: bias forces vanish, so zero torque keeps the state
    x = np.zeros(37)
    x[18] = 0.7
    np.testing.assert_array_equal(orc.dyn(QUAD, p, x, np.zeros(12)), x)
    # response to torque at rest: dv = dt M^-1 S u, so S^T dv/dt is a
    # principal block of an SPD inverse: symmetric and positive definite,
    # with eigenvalues in [1/lambda_max(M), 1/0.9]
    x = np.zeros(37)
    x[:18] = np.random.default_rng(4).uniform(-1, 1, 18)
    base = orc.dyn(QUAD, p, x, np.zeros(12))
    Rm = np.zeros((12, 12))
    for j in range(12):
        u = np.zeros(12)
        u[j] = 1.0
        Rm[:, j] = (orc.dyn(QUAD, p, x, u)[19 + 6:] - base[19 + 6:]) / dt
    assert np.allclose(Rm, Rm.T, atol=1e-12)
    ev = np.linalg.eigvalsh(0.5 * (Rm + Rm.T))
    assert ev.min() > 0 and ev.max() <= 1 / 0.9 + 1e-12
    # the response is linear in u
    u1, u2 = np.random.default_rng(5).normal(size=(2, 12))
    lhs = orc.dyn(QUAD, p, x, u1 + u2) - base
    rhs = (orc.dyn(QUAD, p, x, u1) - base) + (orc.dyn(QUAD, p, x, u2) - base)
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_quad_dynamics_definition(orc):
    # Definitional restatement of the synthetic quadruped (it has no physical
    # identity to check against): M = A^T A + diag(1 + 0.1 sin qb),
    # b = W1 sin qb + (W2 cos qb) * v, v+ = v + dt M^-1 (S u - b), q+ = q + dt E v+.
    p = I.quad_params(1)
    dt = p[0]
    A = p[I.QUAD_OFF_A:I.QUAD_OFF_W1].reshape(18, 18)
    W1 = p[I.QUAD_OFF_W1:I.QUAD_OFF_W2].reshape(18, 18)
    W2 = p[I.QUAD_OFF_W2:I.QUAD_OFF_E].reshape(18, 18)
    e = p[I.QUAD_OFF_E:I.QUAD_OFF_XNOM]
    rng = np.random.default_rng(6)
    x, u = np.r_[rng.uniform(-1, 1, 19), rng.uniform(-1, 1, 18)], rng.normal(size=12)
    q, v = x[:19], x[19:]
    M = A.T @ A + np.diag(1 + 0.1 * np.sin(q[:18]))
    b = W1 @ np.sin(q[:18]) + (W2 @ np.cos(q[:18])) * v
    Su = np.r_[np.zeros(6), u]
    vn = v + dt * np.linalg.solve(M, Su - b)
    E = np.vstack([np.eye(18), e[None, :]])
    np.testing.assert_allclose(orc.dyn(QUAD, p, x, u), np.r_[q + dt * E @ vn, vn], rtol=1e-13, atol=1e-14)
