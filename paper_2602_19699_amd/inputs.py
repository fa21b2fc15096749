"""Seeded synthetic problem data for the batched trajectory-optimization solver.

This module only draws numbers: system parameter vectors, initial states and
horizons.  It holds none of the solver's arithmetic (no dynamics, no costs, no
derivatives), so both the FP64 CPU oracle and the HIP path can consume what it
produces without sharing any computation.

Problem family (paper Sec. II, eq. 1): a finite-horizon discrete-time OCP
    min_{X,U} sum_{k<T} l(x_k,u_k) + l_T(x_T),  x_{k+1} = f(x_k,u_k),  x_0 = x_init,
solved once per sampled initial state (Sec. II, the batch of N TO problems).
The paper's own scenarios (Sec. V-A: point mass, manipulator, target at
[-7,0], elliptical obstacles) are not fully specified in the text, so the
systems below are synthetic stand-ins with the shapes of those workloads.

Parameter-vector layouts are fixed and documented in include/cbic.h; the
offsets here must match that header.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- kinds
SYS_LQ = 0
SYS_POINT_MASS = 1
SYS_PLANAR3 = 2
SYS_QUAD_SYNTH = 3

# ---------------------------------------------------------------- point mass
# [dt, w_u, w_p, w_T, w_obs, g_x, g_y, (c_x, c_y, r) x 3]
PM_NPARAM = 16
PM_N, PM_M = 4, 2


def point_mass_params(seed: int = 0, dt: float = 0.01, w_u: float = 1e-2,
                      w_p: float = 1.0, w_T: float = 10.0,
                      w_obs: float = 1.0) -> np.ndarray:
    """2-D double integrator with a goal and three soft Gaussian obstacles."""
    rng = np.random.default_rng(seed)
    goal = rng.uniform(-2.0, 2.0, 2)
    centres = rng.uniform(-1.5, 1.5, (3, 2))
    radii = rng.uniform(0.2, 0.6, 3)
    p = np.zeros(PM_NPARAM)
    p[0:5] = [dt, w_u, w_p, w_T, w_obs]
    p[5:7] = goal
    for i in range(3):
        p[7 + 3 * i: 10 + 3 * i] = [centres[i, 0], centres[i, 1], radii[i]]
    return p


def point_mass_x0(B: int, seed: int = 1001) -> np.ndarray:
    """Initial states uniform in [-2,2]^2 x [-0.5,0.5]^2, shape (B, 4)."""
    rng = np.random.default_rng(seed)
    lo = np.array([-2.0, -2.0, -0.5, -0.5])
    hi = -lo
    return rng.uniform(lo, hi, (B, 4))


# ---------------------------------------------------------------- planar 3-link arm
# [dt, m1, m2, m3, l1, l2, l3, w_u, w_ee, w_T, w_obs, p_x, p_y, c_x, c_y, r]
P3_NPARAM = 16
P3_N, P3_M = 6, 3


def planar3_params(seed: int = 0, dt: float = 0.01, w_u: float = 1e-2,
                   w_ee: float = 1.0, w_T: float = 10.0,
                   w_obs: float = 1.0) -> np.ndarray:
    """Planar 3-link arm of uniform rods in a horizontal plane."""
    rng = np.random.default_rng(seed)
    masses = rng.uniform(0.5, 2.0, 3)
    lengths = rng.uniform(0.3, 0.8, 3)
    reach = float(lengths.sum())
    rho_t = rng.uniform(0.2, 0.9) * reach
    ang_t = rng.uniform(-np.pi, np.pi)
    rho_c = rng.uniform(0.3, 0.8) * reach
    ang_c = rng.uniform(-np.pi, np.pi)
    r_obs = rng.uniform(0.05, 0.2)
    p = np.zeros(P3_NPARAM)
    p[0] = dt
    p[1:4] = masses
    p[4:7] = lengths
    p[7:11] = [w_u, w_ee, w_T, w_obs]
    p[11:13] = [rho_t * np.cos(ang_t), rho_t * np.sin(ang_t)]
    p[13:15] = [rho_c * np.cos(ang_c), rho_c * np.sin(ang_c)]
    p[15] = r_obs
    return p


def planar3_x0(B: int, seed: int = 1003) -> np.ndarray:
    """Joint angles uniform in [-pi,pi]^3, joint rates in [-0.5,0.5]^3."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(-np.pi, np.pi, (B, 3))
    qd = rng.uniform(-0.5, 0.5, (B, 3))
    return np.concatenate([q, qd], axis=1)


def horizons(B: int, lo: int, hi: int, seed: int = 2003) -> np.ndarray:
    """Per-instance horizons uniform on the integers lo..hi (inclusive)."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, B).astype(np.int32)


# ---------------------------------------------------------------- synthetic quadruped
# [dt, w_u, w_T, w_q, w_v, A(18x18), W1(18x18), W2(18x18), e(18), x_nom(37)]
QUAD_NQ, QUAD_NV, QUAD_M = 19, 18, 12
QUAD_N = QUAD_NQ + QUAD_NV
QUAD_OFF_A = 5
QUAD_OFF_W1 = QUAD_OFF_A + 18 * 18
QUAD_OFF_W2 = QUAD_OFF_W1 + 18 * 18
QUAD_OFF_E = QUAD_OFF_W2 + 18 * 18
QUAD_OFF_XNOM = QUAD_OFF_E + 18
QUAD_NPARAM = QUAD_OFF_XNOM + QUAD_N


def quad_params(seed: int = 0, dt: float = 0.01, w_u: float = 1e-3,
                w_T: float = 10.0, w_q: float = 1.0,
                w_v: float = 0.1) -> np.ndarray:
    """Quadruped-sized synthetic rigid-body-like system (q in R^19, v in R^18)."""
    rng = np.random.default_rng(seed)
    A = rng.normal(0.0, np.sqrt(1.0 / 18.0), (18, 18))
    W1 = rng.normal(0.0, np.sqrt(0.01 / 18.0), (18, 18))
    W2 = rng.normal(0.0, np.sqrt(0.01 / 18.0), (18, 18))
    e = 0.1 * rng.normal(0.0, 1.0, 18)
    q_nom = rng.uniform(-0.5, 0.5, QUAD_NQ)
    p = np.zeros(QUAD_NPARAM)
    p[0:5] = [dt, w_u, w_T, w_q, w_v]
    p[QUAD_OFF_A:QUAD_OFF_W1] = A.ravel()
    p[QUAD_OFF_W1:QUAD_OFF_W2] = W1.ravel()
    p[QUAD_OFF_W2:QUAD_OFF_E] = W2.ravel()
    p[QUAD_OFF_E:QUAD_OFF_XNOM] = e
    p[QUAD_OFF_XNOM:QUAD_OFF_XNOM + QUAD_NQ] = q_nom
    return p


def quad_x0(B: int, params: np.ndarray, seed: int = 1004) -> np.ndarray:
    """q = q_nom + U(-0.5,0.5), v ~ U(-0.5,0.5); shape (B, 37)."""
    rng = np.random.default_rng(seed)
    q_nom = params[QUAD_OFF_XNOM:QUAD_OFF_XNOM + QUAD_NQ]
    q = q_nom[None, :] + rng.uniform(-0.5, 0.5, (B, QUAD_NQ))
    v = rng.uniform(-0.5, 0.5, (B, QUAD_NV))
    return np.concatenate([q, v], axis=1)


# ---------------------------------------------------------------- linear-quadratic
def lq_params(A, B, Q, R, QT, x_ref=None) -> np.ndarray:
    """Pack [n, m, A, B, Q, R, Q_T, x_ref] (row-major) for the LQ kind."""
    A = np.asarray(A, float)
    Bm = np.asarray(B, float)
    n, m = Bm.shape
    x_ref = np.zeros(n) if x_ref is None else np.asarray(x_ref, float)
    return np.concatenate([[float(n), float(m)], A.ravel(), Bm.ravel(),
                           np.asarray(Q, float).ravel(),
                           np.asarray(R, float).ravel(),
                           np.asarray(QT, float).ravel(), x_ref])


def lq_random(n: int, m: int, seed: int = 0, ref: bool = False) -> np.ndarray:
    """A random stabilisable LQ problem with SPD weights (spectrum >= 0.1)."""
    rng = np.random.default_rng(seed)
    A = np.eye(n) + 0.05 * rng.normal(size=(n, n))
    Bm = 0.1 * rng.normal(size=(n, m))

    def spd(k, lo):
        G = rng.normal(size=(k, k))
        return G @ G.T / k + lo * np.eye(k)

    Q, R, QT = spd(n, 0.1), spd(m, 0.1), spd(n, 0.5)
    x_ref = rng.normal(size=n) if ref else None
    return lq_params(A, Bm, Q, R, QT, x_ref)


def lq_x0(B: int, n: int, seed: int = 1000) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (B, n))


# ---------------------------------------------------------------- networks
def mlp_param_count(in_dim: int, width: int, depth: int, out_dim: int) -> int:
    return in_dim * width + width + (depth - 1) * (width * width + width) + width * out_dim + out_dim


def mlp_params(in_dim: int, width: int, depth: int, out_dim: int, seed: int = 0,
               bias_std: float = 0.1) -> np.ndarray:
    """Random-initialised perceptron parameters in the packed layout of the
    library (W_0, b_0, ..., W_out, b_out; row-major, y = x W + b), FP32:
    weights N(0, 1/fan_in) (LeCun normal, the usual default of the paper's
    network library), biases N(0, bias_std^2) so that the bias paths matter.
    Stand-ins for trained networks, which the paper does not publish."""
    rng = np.random.default_rng(seed)
    parts = []
    fan = in_dim
    for _ in range(depth):
        parts += [rng.normal(0.0, 1.0 / np.sqrt(fan), (fan, width)).ravel(), rng.normal(0.0, bias_std, width)]
        fan = width
    parts += [rng.normal(0.0, 1.0 / np.sqrt(fan), (fan, out_dim)).ravel(), rng.normal(0.0, bias_std, out_dim)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == mlp_param_count(in_dim, width, depth, out_dim)
    return out


def bic_candidates(name: str, Bc: int, seed: int = 3001):
    """Candidate initial states of the biased selection (Sec. III-D): draws
    from the workload's initial-state distribution, each with a random start
    s uniform on 0..T_max-1 steps into the episode, i.e. a remaining horizon
    T = T_max - s.  Returns (x [Bc][n], T [Bc] int32, T_max)."""
    kind, params, _, T_max, _ = workload(name, B=1)
    if kind == SYS_POINT_MASS:
        x = point_mass_x0(Bc, seed)
    elif kind == SYS_PLANAR3:
        x = planar3_x0(Bc, seed)
    else:
        raise ValueError("candidates are drawn for the point mass and the arm")
    rng = np.random.default_rng(seed + 1)
    steps = rng.integers(0, T_max, Bc)
    return x, (T_max - steps).astype(np.int32), T_max


# ---------------------------------------------------------------- workloads
def workload(name: str, B: int | None = None, sys_seed: int = 0):
    """Return (kind, params, x0, T_max, T_per_instance or None) for a named workload.

    Names: 'pm64' (point mass, 64 instances, T=100), 'pm16k' (16384 instances),
    'arm4k' (3-link arm, 4096 instances, T uniform 50..200),
    'quad1k' (synthetic quadruped, 1024 instances, T=100).
    """
    if name in ("pm64", "pm16k"):
        B = B or (64 if name == "pm64" else 16384)
        p = point_mass_params(sys_seed)
        return SYS_POINT_MASS, p, point_mass_x0(B, 1001 if name == "pm64" else 1002), 100, None
    if name == "arm4k":
        B = B or 4096
        p = planar3_params(sys_seed)
        return SYS_PLANAR3, p, planar3_x0(B), 200, horizons(B, 50, 200)
    if name == "quad1k":
        B = B or 1024
        p = quad_params(sys_seed)
        return SYS_QUAD_SYNTH, p, quad_x0(B, p), 100, None
    raise ValueError(f"unknown workload {name!r}")
