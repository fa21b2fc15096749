"""Pins of the oracle's iLQR solve: the linear-quadratic closed form, brute
force on tiny horizons, adjoint gradients against finite differences,
monotone decrease, the critic-target extraction and the status semantics."""
import json
import os

import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

PM, P3, QUAD, LQ = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_QUAD_SYNTH, I.SYS_LQ
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lq_scalar.json")


def riccati_textbook(A, B, Q, R, QT, T):
    """Finite-horizon discrete Riccati recursion for sum x'Qx + u'Ru + x_T'Q_T x_T."""
    P = QT.copy()
    Ks = [None] * T
    for k in reversed(range(T)):
        S = R + B.T @ P @ B
        K = np.linalg.solve(S, B.T @ P @ A)
        Ks[k] = K
        P = Q + A.T @ P @ A - A.T @ P @ B @ K
        P = 0.5 * (P + P.T)
    return P, Ks


def lq_dense_optimum(A, B, Q, R, QT, xr, x0, T):
    """Optimum of the same LQ problem as one dense QP in U (solved by numpy)."""
    n, m = B.shape
    # X = F x0 + G U  (stacked x_1..x_T)
    F = np.zeros((T * n, n))
    G = np.zeros((T * n, T * m))
    Ak = np.eye(n)
    for k in range(T):
        Ak = A @ Ak
        F[k * n:(k + 1) * n] = Ak
        for j in range(k + 1):
            G[k * n:(k + 1) * n, j * m:(j + 1) * m] = np.linalg.matrix_power(A, k - j) @ B
    Qbar = np.zeros((T * n, T * n))
    for k in range(T - 1):
        Qbar[k * n:(k + 1) * n, k * n:(k + 1) * n] = Q
    Qbar[(T - 1) * n:, (T - 1) * n:] = QT
    Rbar = np.kron(np.eye(T), R)
    r = np.tile(xr, T)
    d = F @ x0 - r
    H = G.T @ Qbar @ G + Rbar
    U = np.linalg.solve(H, -G.T @ Qbar @ d)
    X = F @ x0 + G @ U
    J = (x0 - xr) @ Q @ (x0 - xr) + (X - r) @ Qbar @ (X - r) + U @ Rbar @ U
    return J, U.reshape(T, m)


def unpack_lq(p):
    n, m = int(p[0]), int(p[1])
    c = 2
    A = p[c:c + n * n].reshape(n, n); c += n * n
    B = p[c:c + n * m].reshape(n, m); c += n * m
    Q = p[c:c + n * n].reshape(n, n); c += n * n
    R = p[c:c + m * m].reshape(m, m); c += m * m
    QT = p[c:c + n * n].reshape(n, n); c += n * n
    return A, B, Q, R, QT, p[c:c + n]


def test_lq_scalar_golden(orc):
    g = json.load(open(GOLDEN))
    p = I.lq_params([[g["A"]]], [[g["B"]]], [[g["Q"]]], [[g["R"]]], [[g["QT"]]])
    for c in g["cases"]:
        r = orc.solve_batch(LQ, p, np.array([[c["x0"]]]), c["T"], opts=orc.Options(max_iter=3))
        assert abs(r.J[0] - c["J"]) < 1e-14 * c["J"]
        assert abs(r.U[0, 0, 0] - c["u0"]) < 1e-14
        assert r.iters[0] == 1 and r.jtrace[0, 0] == 0  # one full Newton step, alpha = 1


@pytest.mark.parametrize("n,m,T", [(2, 1, 5), (4, 2, 30), (6, 3, 50)])
def test_lq_one_iteration_reaches_riccati_optimum(orc, n, m, T):
    p = I.lq_random(n, m, seed=n)
    A, B, Q, R, QT, xr = unpack_lq(p)
    x0 = I.lq_x0(8, n)
    rng = np.random.default_rng(3)
    U0 = rng.normal(size=(8, T, m))  # any warm start
    r1 = orc.solve_batch(LQ, p, x0, T, U0=U0, opts=orc.Options(max_iter=1))
    r2 = orc.solve_batch(LQ, p, x0, T, U0=U0, opts=orc.Options(max_iter=2))
    P0, Ks = riccati_textbook(A, B, Q, R, QT, T)
    for b in range(8):
        Jstar = x0[b] @ P0 @ x0[b]  # P0 already holds the stage-0 state cost
        assert abs(r1.J[b] - Jstar) <= 1e-11 * Jstar
        # optimal closed loop u_k = -K_k x_k
        x = x0[b]
        for k in range(T):
            u = -Ks[k] @ x
            np.testing.assert_allclose(r1.U[b, k], u, atol=1e-10)
            x = A @ x + B @ u
        # a second iteration cannot improve beyond rounding
        assert abs(r2.J[b] - r1.J[b]) <= 1e-12 * r1.J[b]


def test_lq_with_reference_matches_dense_qp(orc):
    p = I.lq_random(4, 2, seed=9, ref=True)
    A, B, Q, R, QT, xr = unpack_lq(p)
    T = 12
    x0 = I.lq_x0(4, 4, seed=5)
    r = orc.solve_batch(LQ, p, x0, T, opts=orc.Options(max_iter=2))
    for b in range(4):
        J, U = lq_dense_optimum(A, B, Q, R, QT, xr, x0[b], T)
        assert abs(r.J[b] - J) <= 1e-11 * J
        np.testing.assert_allclose(r.U[b], U, atol=1e-9)


def _grid_min(orc, kind, p, x0, T, m, lo, hi, levels=4, pts=9):
    """Multi-level grid search over U in [lo,hi]^(T m) using the oracle's
    plain rollout cost (a search, not the solver)."""
    centre = np.zeros(T * m)
    half = (hi - lo) / 2
    best = None
    for _ in range(levels):
        axes = [np.linspace(c - half, c + half, pts) for c in centre]
        grid = np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, T * m)
        J = orc.rollout_costs(kind, p, x0, grid.reshape(-1, T, m))
        i = int(np.argmin(J))
        best = (J[i], grid[i])
        centre = grid[i]
        half = half * 2.5 / (pts - 1)
    return best


def test_brute_force_tiny_horizon_convex(orc):
    # point mass with obstacles moved far away: convex in U, so the grid
    # minimum and the iLQR solution agree to grid resolution
    p = I.point_mass_params(0).copy()
    p[0] = 0.3
    p[[7, 8, 10, 11, 13, 14]] = 1e3
    x0 = np.array([[0.5, -0.4, 0.2, 0.1]])
    r = orc.solve_batch(PM, p, x0, 2)
    Jg, _ = _grid_min(orc, PM, p, x0[0], 2, 2, -20.0, 20.0, levels=6)
    assert r.J[0] <= Jg + 1e-9
    assert Jg - r.J[0] <= 1e-4 * r.J[0]


def test_brute_force_tiny_horizon_with_obstacle(orc):
    # one obstacle near the start: iLQR finds a local minimum, never below the
    # grid's global search by more than its resolution
    p = I.point_mass_params(1).copy()
    p[0] = 0.3
    p[4] = 3.0
    p[[7, 8, 9]] = [0.2, 0.0, 0.5]
    p[[10, 11, 13, 14]] = 1e3
    for x0 in ([0.0, 0.1, 0.0, 0.0], [0.5, -0.3, 0.0, 0.2]):
        x0 = np.array([x0])
        r = orc.solve_batch(PM, p, x0, 3)
        Jg, _ = _grid_min(orc, PM, p, x0[0], 3, 2, -15.0, 15.0, levels=8, pts=7)
        assert r.J[0] >= Jg - 1e-4 * Jg  # the refined grid resolves J to ~1e-5


@pytest.mark.parametrize("kind", [PM, P3, QUAD], ids=["pm", "arm", "quad"])
def test_adjoint_gradient_matches_finite_differences(orc, kind):
    p = {PM: I.point_mass_params(0), P3: I.planar3_params(0), QUAD: I.quad_params(0)}[kind]
    n, m = orc.dims(kind, p)
    T = 20
    rng = np.random.default_rng(kind)
    x0 = {PM: lambda: I.point_mass_x0(1)[0], P3: lambda: I.planar3_x0(1)[0],
          QUAD: lambda: I.quad_x0(1, p)[0]}[kind]()
    U = rng.normal(size=(T, m))
    X, J, lam, g = orc.gradient(kind, p, x0, U)
    h = 1e-6
    idx = [(k, i) for k in (0, 7, T - 1) for i in range(min(m, 3))]
    for k, i in idx:
        Up, Um = U.copy(), U.copy()
        Up[k, i] += h
        Um[k, i] -= h
        Jp, Jm = orc.rollout_costs(kind, p, x0, np.stack([Up, Um]))
        assert abs((Jp - Jm) / (2 * h) - g[k, i]) <= 1e-6 * max(1.0, abs(g[k, i]))
    for i in range(min(n, 4)):
        e = np.zeros(n)
        e[i] = h
        Jp, Jm = orc.rollout_costs(kind, p, x0 + e, U[None]), orc.rollout_costs(kind, p, x0 - e, U[None])
        assert abs((Jp[0] - Jm[0]) / (2 * h) - lam[0, i]) <= 1e-6 * max(1.0, abs(lam[0, i]))


def test_solution_is_a_local_minimum_and_costs_decrease(orc):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(16)
    r = orc.solve_batch(PM, p, x0, 100)
    rng = np.random.default_rng(0)
    for b in range(16):
        acc = r.trace[b, : r.iters[b] + 1]
        assert np.all(np.diff(acc) < 0)  # every accepted step strictly lowers J
        _, J, _, g = orc.gradient(PM, p, x0[b], r.U[b])
        assert J == r.J[b]
        assert np.abs(g).max() < 1e-5 * (1 + np.abs(r.U[b]).max())
        Up = r.U[b][None] + 1e-4 * rng.normal(size=(64, 100, 2))
        assert orc.rollout_costs(PM, p, x0[b], Up).min() >= r.J[b] - 1e-12 * r.J[b]


def test_extraction_targets(orc):
    p = I.planar3_params(0)
    B, Tmax = 6, 60
    x0 = I.planar3_x0(B)
    T = np.array([60, 17, 33, 1, 2, 45], np.int32)
    for K in (0, 1, 5, 60, 100):
        r = orc.solve_batch(P3, p, x0, Tmax, T=T, opts=orc.Options(max_iter=8, lookahead=K))
        for b in range(B):
            Tb, Kb = T[b], (T[b] if K <= 0 else K)
            X, U = r.X[b, :Tb + 1], r.U[b, :Tb]
            c = [orc.cost(P3, p, X[k], U[k]) for k in range(Tb)] + [orc.term(P3, p, X[Tb])]
            V = r.Vbar[b]
            assert V[Tb] == c[Tb]
            if Kb >= Tb:
                assert abs(V[0] - r.J[b]) <= 1e-13 * r.J[b]
            for k in range(Tb):  # one-step telescoping of the window sum
                nxt = V[k + 1] if k + 1 <= Tb else 0.0
                leave = (c[k + Kb] if k + Kb < Tb else 0.0) + (c[Tb] if k + Kb == Tb - 1 else 0.0)
                if k + Kb >= Tb:
                    leave = 0.0
                assert abs(V[k] - (c[k] + nxt - leave)) <= 1e-12 * max(1.0, V[k])
            for k in range(Tb + 1):
                np.testing.assert_array_equal(r.xK[b, k], X[min(k + Kb, Tb)])
            assert np.all(r.Vbar[b, Tb + 1:] == 0) and np.all(r.X[b, Tb + 1:] == 0)
        # costate = gradient of the full tail cost w.r.t. the state (U fixed)
        b, k, h = 0, 10, 1e-6
        for i in range(6):
            e = np.zeros(6)
            e[i] = h
            Jp = orc.rollout_costs(P3, p, r.X[b, k] + e, r.U[b, k:T[b]][None])[0]
            Jm = orc.rollout_costs(P3, p, r.X[b, k] - e, r.U[b, k:T[b]][None])[0]
            assert abs((Jp - Jm) / (2 * h) - r.Vx[b, k, i]) <= 1e-6 * max(1, abs(r.Vx[b, k, i]))


def test_status_semantics(orc):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(4)
    x0[1, 2] = np.nan
    r = orc.solve_batch(PM, p, x0, 50, opts=orc.Options(max_iter=50))
    assert r.status[1] == orc.ST_NONFINITE and r.iters[1] == 0
    assert all(r.status[b] == orc.ST_LS_FAILED for b in (0, 2, 3))
    # no trials allowed: the line search fails at once and the warm start stays
    r = orc.solve_batch(PM, p, x0[[0]], 50, opts=orc.Options(ls_trials=0))
    assert r.status[0] == orc.ST_LS_FAILED and r.iters[0] == 0
    assert np.all(r.U == 0)
    # iteration cap
    r = orc.solve_batch(PM, p, x0[[0]], 50, opts=orc.Options(max_iter=1))
    assert r.status[0] == orc.ST_MAX_ITER and r.iters[0] == 1
    # tolerance mode
    r = orc.solve_batch(PM, p, x0[[0]], 50, opts=orc.Options(stop_mode=1, rtol=1e-6))
    assert r.status[0] == orc.ST_CONVERGED
    # indefinite control Hessian clipped to zero with eps = 0 and no control
    # authority: Q_uu is singular and its Cholesky fails
    lq = I.lq_params(np.eye(2), np.zeros((2, 1)), np.eye(2), -np.eye(1), np.eye(2))
    r = orc.solve_batch(LQ, lq, np.ones((1, 2)), 5, opts=orc.Options(eps=0.0))
    assert r.status[0] == orc.ST_CHOL_FAIL and r.iters[0] == 0


def test_batch_independence_ragged_and_resume(orc):
    p = I.planar3_params(0)
    x0 = I.planar3_x0(5)
    T = np.array([30, 12, 30, 7, 25], np.int32)
    o = orc.Options(max_iter=12)
    rb = orc.solve_batch(P3, p, x0, 30, T=T, opts=o)
    for b in range(5):
        ra = orc.solve_batch(P3, p, x0[[b]], int(T[b]), opts=o)
        assert ra.J[0] == rb.J[b]
        np.testing.assert_array_equal(ra.X[0], rb.X[b, :T[b] + 1])
    # resume: 5 iterations, then 7 more from the returned controls, equals 12
    r5 = orc.solve_batch(P3, p, x0, 30, T=T, opts=orc.Options(max_iter=5))
    r7 = orc.solve_batch(P3, p, x0, 30, T=T, U0=r5.U, opts=orc.Options(max_iter=7))
    for b in range(5):
        if r5.status[b] & orc.ST_MAX_ITER:
            assert r7.J[b] == rb.J[b]
