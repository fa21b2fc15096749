"""ctypes binding of the FP64 CPU oracle (oracle.cpp).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the solver library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import dataclasses
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

ST_CONVERGED, ST_MAX_ITER, ST_LS_FAILED, ST_NONFINITE, ST_CHOL_FAIL = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-Wall", "-o", LIB + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Opts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("ls_trials", C.c_int32),
                ("stop_mode", C.c_int32), ("lookahead", C.c_int32),
                ("eps", C.c_double), ("beta", C.c_double), ("rtol", C.c_double),
                ("reg", C.c_int32), ("mu0", C.c_double), ("mu_factor", C.c_double),
                ("mu_max", C.c_double), ("umax", C.c_double), ("round32", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Options:
    max_iter: int = 50
    ls_trials: int = 16
    stop_mode: int = 0
    lookahead: int = 0
    eps: float = 1e-6
    beta: float = 0.5
    rtol: float = 1e-10
    # regularisation of the backward pass: 0 = eigenvalue clipping (eq. 7),
    # 1 = Levenberg-Marquardt (Sec. IV-B ablation: no clipping, Q_uu + mu I)
    reg: int = 0
    mu0: float = 1e-6
    mu_factor: float = 10.0
    mu_max: float = 1e10
    # control bound |u_k,i| <= umax of eq. 1 (infinite: unbounded)
    umax: float = float("inf")
    # sensitivity probe for the mixed-precision form, off by default: round
    # what that form keeps in FP32 (states, controls, derivative blocks,
    # clipped Hessians, P and p, gains) to FP32 where it is produced
    round32: int = 0

    def c(self):
        return _Opts(self.max_iter, self.ls_trials, self.stop_mode, self.lookahead,
                     self.eps, self.beta, self.rtol, self.reg, self.mu0, self.mu_factor,
                     self.mu_max, self.umax, self.round32)


def dims(kind, params):
    params = _f64(params)
    n, m = C.c_int(), C.c_int()
    if lib().orc_dims(kind, _p(params), len(params), C.byref(n), C.byref(m)) != 0:
        raise ValueError("bad system kind / parameter vector")
    return n.value, m.value


def dyn(kind, params, x, u):
    params = _f64(params)
    n, _ = dims(kind, params)
    out = np.zeros(n)
    lib().orc_dyn(kind, _p(params), len(params), _p(_f64(x)), _p(_f64(u)), _p(out))
    return out


def dyn_jac(kind, params, x, u):
    params = _f64(params)
    n, m = dims(kind, params)
    A, B = np.zeros((n, n)), np.zeros((n, m))
    lib().orc_dyn_jac(kind, _p(params), len(params), _p(_f64(x)), _p(_f64(u)), _p(A), _p(B))
    return A, B


def cost(kind, params, x, u):
    params = _f64(params)
    out = C.c_double()
    lib().orc_cost(kind, _p(params), len(params), _p(_f64(x)), _p(_f64(u)), C.byref(out))
    return out.value


def cost_derivs(kind, params, x, u):
    params = _f64(params)
    n, m = dims(kind, params)
    lx, lu = np.zeros(n), np.zeros(m)
    lxx, luu, lux = np.zeros((n, n)), np.zeros((m, m)), np.zeros((m, n))
    lib().orc_cost_derivs(kind, _p(params), len(params), _p(_f64(x)), _p(_f64(u)),
                          _p(lx), _p(lu), _p(lxx), _p(luu), _p(lux))
    return lx, lu, lxx, luu, lux


def term(kind, params, x):
    params = _f64(params)
    out = C.c_double()
    lib().orc_term(kind, _p(params), len(params), _p(_f64(x)), C.byref(out))
    return out.value


def term_derivs(kind, params, x):
    params = _f64(params)
    n, _ = dims(kind, params)
    lx, lxx = np.zeros(n), np.zeros((n, n))
    lib().orc_term_derivs(kind, _p(params), len(params), _p(_f64(x)), _p(lx), _p(lxx))
    return lx, lxx


def box_qp(H, g, lo, hi):
    """Bounded control step: (d, held) minimising 0.5 d'Hd + g'd over lo <= d <= hi
    (the oracle's active-set solver, started from the unconstrained minimiser)."""
    H, g, lo, hi = _f64(H), _f64(g), _f64(lo), _f64(hi)
    m = len(g)
    d = -np.linalg.solve(H, g)
    held = np.zeros(m, np.int32)
    if lib().orc_box_qp(m, _p(H), _p(g), _p(lo), _p(hi), _p(d), held.ctypes.data_as(C.c_void_p)) != 0:
        raise ValueError("a face of H does not factorise")
    return d, held.astype(bool)


def psd_clip(H, eps):
    H = _f64(H)
    out = np.zeros_like(H)
    lib().orc_psd_clip(H.shape[0], _p(H), C.c_double(eps), _p(out))
    return out


def eig(H):
    H = _f64(H)
    n = H.shape[0]
    S, W = np.zeros(n), np.zeros((n, n))
    lib().orc_eig(n, _p(H), _p(S), _p(W))
    return S, W


def p3_mass(params, q):
    M = np.zeros((3, 3))
    lib().orc_p3_mass(_p(_f64(params)), _p(_f64(q)), _p(M))
    return M


def p3_ee(params, q):
    ee = np.zeros(2)
    lib().orc_p3_ee(_p(_f64(params)), _p(_f64(q)), _p(ee))
    return ee


def rollout_costs(kind, params, x0, U, nthreads=0):
    """Total cost of each control sequence in U (nb, T, m) from one x0."""
    params = _f64(params)
    U = _f64(U)
    nb, T = U.shape[0], U.shape[1]
    J = np.zeros(nb)
    lib().orc_rollout_costs(kind, _p(params), len(params), T, _p(_f64(x0)), nb, _p(U), _p(J),
                            nthreads)
    return J


def gradient(kind, params, x0, U):
    """(X, J, lambda, dJ/dU) along the rollout of U from x0."""
    params = _f64(params)
    U = _f64(U)
    n, m = dims(kind, params)
    T = U.shape[0]
    X, lam, g = np.zeros((T + 1, n)), np.zeros((T + 1, n)), np.zeros((T, m))
    J = C.c_double()
    lib().orc_gradient(kind, _p(params), len(params), T, _p(_f64(x0)), _p(U), _p(X),
                       C.byref(J), _p(lam), _p(g))
    return X, J.value, lam, g


@dataclass
class Result:
    X: np.ndarray
    U: np.ndarray
    J: np.ndarray
    iters: np.ndarray
    status: np.ndarray
    Vbar: np.ndarray
    Vx: np.ndarray
    xK: np.ndarray
    trace: np.ndarray
    jtrace: np.ndarray
    margin: np.ndarray


def solve_batch(kind, params, x0, T_max, T=None, U0=None, opts: Options | None = None,
                force_j=None, nthreads=0) -> Result:
    """Solve every instance (rows of x0) on the CPU in FP64."""
    opts = opts or Options()
    params = _f64(params)
    x0 = _f64(x0)
    n, m = dims(kind, params)
    B = x0.shape[0]
    Tb = None if T is None else np.ascontiguousarray(T, dtype=np.int32)
    U0c = None if U0 is None else _f64(U0).reshape(B, T_max, m)
    fj = None if force_j is None else np.ascontiguousarray(force_j, dtype=np.int32)
    X = np.zeros((B, T_max + 1, n))
    U = np.zeros((B, T_max, m))
    J = np.zeros(B)
    iters = np.zeros(B, np.int32)
    status = np.zeros(B, np.uint32)
    Vbar = np.zeros((B, T_max + 1))
    Vx = np.zeros((B, T_max + 1, n))
    xK = np.zeros((B, T_max + 1, n))
    trace = np.zeros((B, opts.max_iter + 1))
    jtrace = np.zeros((B, max(opts.max_iter, 1)), np.int32)
    margin = np.zeros((B, max(opts.max_iter, 1)))
    o = opts.c()
    rc = lib().orc_solve_batch(kind, _p(params), len(params), B, T_max, _p(Tb), _p(x0), _p(U0c),
                               C.byref(o), _p(X), _p(U), _p(J), _p(iters), _p(status), _p(Vbar),
                               _p(Vx), _p(xK), _p(trace), _p(jtrace), _p(margin), _p(fj),
                               nthreads)
    if rc != 0:
        lib().orc_last_error.restype = C.c_char_p
        raise ValueError(lib().orc_last_error().decode())
    return Result(X, U, J, iters, status, Vbar, Vx, xK, trace, jtrace, margin)


def max_threads() -> int:
    return lib().orc_max_threads()


def percentile_nearest_rank(values, q):
    """Nearest-rank percentile: the smallest value v with at least q percent of
    the values <= v (the rank is ceil(q n / 100))."""
    v = sorted(int(x) for x in values)
    rank = -(-q * len(v) // 100)
    return v[max(rank, 1) - 1]


def calibrate_max_iter(kind, params, x0, T_max, T=None, opts: Options | None = None, cap=1000, nthreads=0):
    """Iteration budget (paper Sec. IV-A): solve with the relative-decrease stop
    under `cap` iterations and return (p99, p50, counts), the 99th and 50th
    nearest-rank percentiles of the per-instance iteration counts (the oracle
    rejects invalid horizons outright)."""
    base = opts or Options()
    o = dataclasses.replace(base, max_iter=cap, stop_mode=1)
    r = solve_batch(kind, params, x0, T_max, T=T, opts=o, nthreads=nthreads)
    counts = r.iters.astype(np.int64)
    return percentile_nearest_rank(counts, 99), percentile_nearest_rank(counts, 50), counts


@dataclass
class Net:
    """A perceptron as the library describes it (cbic_mlp): FP32 parameters,
    depth hidden layers of `width` units, activation act (0 tanh, 1 ELU,
    2 ReLU), output map out_act (0 identity, 1 out_scale * tanh, 2 softplus)."""
    in_dim: int
    width: int
    depth: int
    out_dim: int
    act: int
    out_act: int
    out_scale: float
    params: np.ndarray  # float32

    def _args(self):
        self.params = np.ascontiguousarray(self.params, dtype=np.float32)
        return (self.in_dim, self.width, self.depth, self.out_dim, self.act, self.out_act,
                C.c_double(self.out_scale), self.params.ctypes.data_as(C.c_void_p))


def mlp_forward(net: Net, x):
    """net(x) for rows x [B][in_dim], in FP64."""
    x = _f64(x)
    B = x.shape[0]
    y = np.zeros((B, net.out_dim))
    if lib().orc_mlp_forward(*net._args(), B, _p(x), _p(y)) != 0:
        raise ValueError("bad network")
    return y


def top_n(scores, N):
    """The N highest scores' indices in ascending index order (Sec. III-D: the N
    most uncertain candidates): ranking by score, higher first, equal scores by
    lower index, NaN below everything, -0 equal to +0."""
    s = np.asarray(scores, dtype=np.float64)
    key = np.where(np.isnan(s), -np.inf, s)
    nan_last = np.isnan(s).astype(np.int64)  # NaN after -inf
    order = np.lexsort((np.arange(len(s)), -key, nan_last))
    return np.sort(order[:N]).astype(np.int64)


def bic_select(net: Net, x, T, T_max, N):
    """(scores, selected) of the biased initial-state selection: the std-critic's
    score of every candidate (x_i, tau_i), tau_i = (T_max - T_i) / T_max (a
    candidate with remaining horizon T_i starts T_max - T_i steps into the
    episode), in FP64, and the top-N indices.  T None: the state alone."""
    x = _f64(x)
    if T is None:
        inp = x
    else:
        tau = (T_max - np.asarray(T, dtype=np.float64)) / T_max
        inp = np.concatenate([x, tau[:, None]], axis=1)
    sc = mlp_forward(net, inp)[:, 0]
    return sc, top_n(sc, N)


def actor_rollout(kind, params, net: Net, x0, T_max, T=None):
    """(U, X) of the actor warm start: u_k = actor(x_k, tau_k), tau_k =
    (T_max - T_b + k) / T_max, x_{k+1} = f(x_k, u_k); zero past each horizon."""
    params = _f64(params)
    x0 = _f64(x0)
    n, m = dims(kind, params)
    B = x0.shape[0]
    U = np.zeros((B, T_max, m))
    X = np.zeros((B, T_max + 1, n))
    Tb = None if T is None else np.ascontiguousarray(T, dtype=np.int32)
    r = lib().orc_actor_rollout(kind, _p(params), len(params), *net._args(), B, T_max,
                                None if Tb is None else Tb.ctypes.data_as(C.c_void_p), _p(x0), _p(U), _p(X))
    if r != 0:
        raise ValueError("bad system or network")
    return U, X


def extract(kind, params, X, U, lookahead=0):
    """(V-bar, V-bar_x, x_K) of the given trajectory X (T+1, n), U (T, m)."""
    params = _f64(params)
    X, U = _f64(X), _f64(U)
    T, n = U.shape[0], X.shape[1]
    Vb, Vx, xK = np.zeros(T + 1), np.zeros((T + 1, n)), np.zeros((T + 1, n))
    if lib().orc_extract(kind, _p(params), len(params), T, _p(X), _p(U), lookahead, _p(Vb), _p(Vx), _p(xK)) != 0:
        raise ValueError("bad arguments")
    return Vb, Vx, xK


def check_trajectory(kind, params, X, U):
    """(max per-step relative dynamics residual, total cost) of a given trajectory."""
    params = _f64(params)
    X, U = _f64(X), _f64(U)
    d, J = C.c_double(), C.c_double()
    lib().orc_check_trajectory(kind, _p(params), len(params), U.shape[0], _p(X), _p(U), C.byref(d), C.byref(J))
    return d.value, J.value
