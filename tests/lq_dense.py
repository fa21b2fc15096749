"""The linear-quadratic problem of the LQ system kind written as one dense
quadratic program in the stacked controls U = (u_0, ..., u_{T-1}), built by
numpy from (A, B, Q, R, Q_T, x_ref) without any recursion: the reference the
LQ pins compare the oracle's iLQR against."""
import numpy as np
from scipy.optimize import lsq_linear


def unpack_lq(p):
    n, m = int(p[0]), int(p[1])
    c = 2
    A = p[c:c + n * n].reshape(n, n); c += n * n
    B = p[c:c + n * m].reshape(n, m); c += n * m
    Q = p[c:c + n * n].reshape(n, n); c += n * n
    R = p[c:c + m * m].reshape(m, m); c += m * m
    QT = p[c:c + n * n].reshape(n, n); c += n * n
    return A, B, Q, R, QT, p[c:c + n]


def dense_qp(p, x0, T):
    """J(U) = sum_k (x_k-r)'Q(x_k-r) + u_k'R u_k + (x_T-r)'Q_T(x_T-r) as
    0.5 U'HU + g0'U + c; returns (H, g0, J)."""
    A, B, Q, R, QT, xr = unpack_lq(p)
    n, m = B.shape
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
    d = F @ x0 - np.tile(xr, T)
    H = 2.0 * (G.T @ Qbar @ G + Rbar)
    g0 = 2.0 * G.T @ Qbar @ d
    c = (x0 - xr) @ Q @ (x0 - xr) + d @ Qbar @ d
    return H, g0, lambda U: 0.5 * U @ H @ U + g0 @ U + c


def bounded_qp(H, g, lo, hi):
    """argmin 0.5 d'Hd + g'd over lo <= d <= hi by SciPy's bounded-variable
    least squares (an exact active-set method): with H = L L',
    0.5 d'Hd + g'd = 0.5 |L'd + L^-1 g|^2 - const."""
    L = np.linalg.cholesky(H)
    b = -np.linalg.solve(L, g)
    r = lsq_linear(L.T, b, bounds=(lo, hi), method="bvls", tol=1e-15, max_iter=1000)
    return r.x
