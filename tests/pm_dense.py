"""The point-mass problem written densely in the stacked controls U =
(u_0, ..., u_{T-1}).  Its dynamics are linear (semi-implicit Euler of a
double integrator: v+ = v + dt u, p+ = p + dt v+), so iLQR's local model is
the exact second-order expansion of J(U) with the cost Hessians replaced as
the iteration prescribes (eigenvalue clip, eq. 7, or plain symmetrisation for
Levenberg-Marquardt), and one iteration's full step is a Newton step on that
dense model.  Built here by numpy from the dynamics' definition and the
oracle's per-step cost derivatives, without the Riccati recursion: the
reference of the line-search and Levenberg-Marquardt pins."""
import numpy as np


def pm_matrices(dt):
    I2, Z2 = np.eye(2), np.zeros((2, 2))
    A = np.block([[I2, dt * I2], [Z2, I2]])
    B = np.vstack([dt * dt * I2, dt * I2])
    return A, B


def rollout(p, x0, U):
    A, B = pm_matrices(p[0])
    X = [np.asarray(x0, float)]
    for u in U:
        X.append(A @ X[-1] + B @ u)
    return np.array(X)


def dense_model(orc, p, x0, U, hess):
    """(g, H): gradient of J at U and the model Hessian, each step's state and
    control cost Hessians mapped through hess (clip or symmetrisation)."""
    from paper_2602_19699_amd import inputs as I
    A, B = pm_matrices(p[0])
    T, m = U.shape
    n = 4
    X = rollout(p, x0, U)
    # G[k] maps U to x_k (k = 1..T): x_k = A^k x0 + sum_{j<k} A^(k-1-j) B u_j
    G = np.zeros((T + 1, n, T * m))
    for k in range(1, T + 1):
        G[k] = A @ G[k - 1]
        G[k][:, (k - 1) * m:k * m] += B
    g = np.zeros(T * m)
    H = np.zeros((T * m, T * m))
    for k in range(T):
        lx, lu, lxx, luu, lux = orc.cost_derivs(I.SYS_POINT_MASS, p, X[k], U[k])
        assert np.all(lux == 0)
        if k > 0:  # x_0 does not depend on U
            g += G[k].T @ lx
            H += G[k].T @ hess(lxx) @ G[k]
        g[k * m:(k + 1) * m] += lu
        H[k * m:(k + 1) * m, k * m:(k + 1) * m] += hess(luu)
    lx, lxx = orc.term_derivs(I.SYS_POINT_MASS, p, X[T])
    g += G[T].T @ lx
    H += G[T].T @ hess(lxx) @ G[T]
    return g, H


def cost(orc, p, x0, U):
    from paper_2602_19699_amd import inputs as I
    return orc.rollout_costs(I.SYS_POINT_MASS, p, x0, U[None])[0]
