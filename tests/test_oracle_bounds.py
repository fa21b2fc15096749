"""Pins of the oracle's control bound |u_k,i| <= u_max (eq. 1): the bounded
control step against SciPy's bounded-variable least squares and the KKT
conditions; the bounded iLQR against the dense bounded QP of linear-quadratic
problems; feasibility and first-order optimality (through the adjoint
gradient) on the point mass."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

from lq_dense import bounded_qp, dense_qp

LQ, PM, P3 = I.SYS_LQ, I.SYS_POINT_MASS, I.SYS_PLANAR3


def _random_box_problem(rng, m):
    G = rng.normal(size=(m, m))
    H = G @ G.T + 0.05 * np.eye(m)
    g = rng.normal(size=m) * 3.0
    u = rng.uniform(-1, 1, size=m)  # the box of the step contains 0: |u| <= 1
    return H, g, -1.0 - u, 1.0 - u


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_box_step_matches_bvls_and_kkt(orc, m):
    rng = np.random.default_rng(40 + m)
    active = 0
    for _ in range(300):
        H, g, lo, hi = _random_box_problem(rng, m)
        d, held = orc.box_qp(H, g, lo, hi)
        ref = bounded_qp(H, g, lo, hi)
        np.testing.assert_allclose(d, ref, atol=1e-10 * (1 + np.abs(ref).max()), rtol=0)
        assert np.all(d >= lo) and np.all(d <= hi)
        # KKT: zero gradient on free components, outward gradient on held ones
        gr = H @ d + g
        scale = 1e-9 * (np.abs(g).max() + np.abs(H).max())
        at_lo, at_hi = held & (d == lo), held & (d == hi)
        assert np.all(held == (at_lo | at_hi))
        assert np.all(np.abs(gr[~held]) <= scale)
        assert np.all(gr[at_lo] >= -scale) and np.all(gr[at_hi] <= scale)
        active += held.any()
    assert active > 50  # the draws exercise the bound


def test_box_step_special_cases(orc):
    # one dimension: the clamped Newton step
    for h, g, lo, hi in [(2.0, 5.0, -1.0, 1.0), (2.0, -5.0, -1.0, 1.0), (2.0, 1.0, -1.0, 1.0)]:
        d, held = orc.box_qp([[h]], [g], [lo], [hi])
        assert d[0] == min(max(-g / h, lo), hi) and held[0] == (abs(g / h) > 1.0)
    # diagonal H: componentwise clamping of the Newton step
    h = np.array([1.0, 4.0, 0.5])
    g = np.array([3.0, -0.5, -2.0])
    lo, hi = np.full(3, -1.0), np.full(3, 1.0)
    d, held = orc.box_qp(np.diag(h), g, lo, hi)
    np.testing.assert_array_equal(d, np.clip(-g / h, lo, hi))
    np.testing.assert_array_equal(held, [True, False, True])
    # inside the box: the unconstrained step, untouched
    H = np.array([[2.0, 0.5], [0.5, 1.0]])
    g = np.array([0.1, -0.2])
    d, held = orc.box_qp(H, g, [-1, -1], [1, 1])
    np.testing.assert_array_equal(d, -np.linalg.solve(H, g))
    assert not held.any()
    # coupling moves a component that is free without the other bound: the
    # clamped Newton step is not the answer
    H = np.array([[1.0, 0.9], [0.9, 1.0]])
    g = np.array([-3.0, 0.0])
    d, held = orc.box_qp(H, g, [-1, -1], [1, 1])
    np.testing.assert_allclose(d, bounded_qp(H, g, np.array([-1.0, -1.0]), np.array([1.0, 1.0])), atol=1e-14)
    np.testing.assert_allclose(d, [1.0, -0.9], atol=1e-15)


def _lq_case(seed, n=4, m=2):
    return I.lq_random(n, m, seed=seed, ref=True)


def test_bounded_lq_one_step_is_the_bounded_qp(orc):
    # T = 1: the bounded iLQR step is the minimiser of the (quadratic) cost over the box
    p = _lq_case(3)
    x0 = I.lq_x0(6, 4, seed=8) * 4.0
    umax = 0.4
    r = orc.solve_batch(LQ, p, x0, 1, opts=orc.Options(max_iter=1, umax=umax))
    held_any = 0
    for b in range(6):
        H, g0, J = dense_qp(p, x0[b], 1)
        u = bounded_qp(H, g0, np.full(2, -umax), np.full(2, umax))
        np.testing.assert_allclose(r.U[b, 0], u, atol=1e-12, rtol=0)
        assert abs(r.J[b] - J(u)) <= 1e-12 * abs(J(u))
        held_any += np.any(np.abs(u) == umax)
    assert held_any >= 3


@pytest.mark.parametrize("umax", [0.15, 0.5])
def test_bounded_lq_converges_to_the_bounded_qp(orc, umax):
    p = _lq_case(9)
    T = 12
    x0 = I.lq_x0(4, 4, seed=5) * 3.0
    r = orc.solve_batch(LQ, p, x0, T, opts=orc.Options(max_iter=100, stop_mode=1, rtol=1e-15, umax=umax))
    active = 0
    for b in range(4):
        H, g0, J = dense_qp(p, x0[b], T)
        u = bounded_qp(H, g0, np.full(T * 2, -umax), np.full(T * 2, umax))
        assert abs(r.J[b] - J(u)) <= 1e-11 * abs(J(u))
        np.testing.assert_allclose(r.U[b].ravel(), u, atol=1e-6, rtol=0)
        assert np.all(np.abs(r.U[b]) <= umax)
        active += np.sum(np.isclose(np.abs(u), umax, rtol=0, atol=1e-12))
    assert active > 0


def test_loose_bound_changes_nothing(orc):
    # a bound that never binds gives the unbounded solve bit for bit
    kind, p, x0, T, _ = I.workload("pm64")
    x0 = x0[:16]
    a = orc.solve_batch(kind, p, x0, T, opts=orc.Options(max_iter=20))
    b = orc.solve_batch(kind, p, x0, T, opts=orc.Options(max_iter=20, umax=1e30))
    for f in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


def test_warm_start_is_clamped(orc):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(3, seed=4)
    T = 20
    U0 = np.random.default_rng(2).normal(size=(3, T, 2)) * 10.0
    r = orc.solve_batch(PM, p, x0, T, U0=U0, opts=orc.Options(max_iter=0, umax=5.0))
    Uc = np.clip(U0, -5.0, 5.0)
    np.testing.assert_array_equal(r.U, Uc)
    for b in range(3):
        assert r.J[b] == orc.rollout_costs(PM, p, x0[b], Uc[b:b + 1])[0]


@pytest.mark.parametrize("kind,umax", [(PM, 10.0), (P3, 8.0)], ids=["pm", "arm"])
def test_bounded_solution_is_feasible_and_stationary(orc, kind, umax):
    if kind == PM:
        p, x0, T, Tb = I.point_mass_params(0), I.point_mass_x0(12, seed=3), 100, None
    else:
        p, x0, T, Tb = I.planar3_params(0), I.planar3_x0(8, seed=6), 120, I.horizons(8, 60, 120, seed=2)
    r = orc.solve_batch(kind, p, x0, T, T=Tb, opts=orc.Options(max_iter=400, stop_mode=1, rtol=1e-13, umax=umax))
    saturated = 0
    for b in range(len(x0)):
        Tb_ = T if Tb is None else int(Tb[b])
        U = r.U[b, :Tb_]
        assert np.all(np.abs(U) <= umax)
        # first-order optimality over the box through the adjoint gradient
        # (pinned against finite differences): zero on interior components,
        # pointing out of the box on components at a bound
        g = orc.gradient(kind, p, x0[b], U)[3]
        tol = 1e-4 * max(1.0, abs(r.J[b]))
        at_hi, at_lo = U >= umax, U <= -umax
        inner = ~(at_hi | at_lo)
        assert np.all(np.abs(g[inner]) <= tol), f"#{b}: interior gradient {np.abs(g[inner]).max():.2e}"
        assert np.all(g[at_hi] <= tol) and np.all(g[at_lo] >= -tol)
        saturated += (at_hi | at_lo).any()
    assert saturated >= len(x0) // 2
