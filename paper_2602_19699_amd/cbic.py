"""Python binding of the C ABI in include/cbic.h (argument marshalling only).

Every step of the solve runs in the HIP kernels of libcbic.so; PyTorch is used
here only to hold device memory and to name the stream.  If the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbic.so")

OK, NOT_READY = 0, 1
E_INVALID, E_OOM, E_HIP, E_BUSY, E_UNSUPPORTED = -1, -2, -3, -4, -5
ST_CONVERGED, ST_MAX_ITER, ST_LS_FAILED, ST_NONFINITE, ST_CHOL_FAIL, ST_BAD_INPUT = 1, 2, 4, 8, 16, 32
SYS_LQ, SYS_POINT_MASS, SYS_PLANAR3, SYS_QUAD_SYNTH = 0, 1, 2, 3
FP64, MIXED = 0, 1
SCHED_AUTO, SCHED_LANE, SCHED_GROUP = 0, 1, 2
REG_CLIP, REG_LM = 0, 1
FLAG_GRAPH = 1
FLAG_TIMING = 2
FLAG_INPUT_ORDER = 4


class CbicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cbic error {code}: {msg}")
        self.code = code


class _Opts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("max_iter", C.c_int32), ("psd_eps", C.c_double),
                ("ls_max_trials", C.c_int32), ("ls_beta", C.c_double), ("stop_mode", C.c_int32),
                ("rtol", C.c_double), ("lookahead_K", C.c_int32), ("precision", C.c_int32),
                ("schedule", C.c_int32), ("iters_per_launch", C.c_int32), ("group_lanes", C.c_int32),
                ("flags", C.c_uint32), ("regularization", C.c_int32), ("lm_mu0", C.c_double),
                ("lm_factor", C.c_double), ("lm_mu_max", C.c_double), ("u_max", C.c_double),
                ("wg_per_cu", C.c_int32)]


class _Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("X", "U", "J", "iters", "status", "Vbar", "Vx", "xK",
                                            "cost_trace", "work", "jtrace")]


class _ServerOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("mem_cap_bytes", C.c_size_t), ("slots_per_class", C.c_int32),
                ("t_max", C.c_int32), ("iters_per_launch", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [("X", C.c_void_p), ("U", C.c_void_p), ("Vbar", C.c_void_p), ("Vx", C.c_void_p),
                ("J", C.c_double), ("iters", C.c_int32), ("status", C.c_uint32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("rounds", C.c_uint64),
                ("inflight_bytes", C.c_size_t), ("peak_inflight_bytes", C.c_size_t), ("pool_bytes", C.c_size_t),
                ("classes", C.c_int32), ("max_resident", C.c_int32), ("peak_pool_bytes", C.c_size_t),
                ("evictions", C.c_uint64), ("launches", C.c_uint64), ("launched_slots", C.c_uint64),
                ("host_busy_s", C.c_double)]


class _Mlp(C.Structure):
    _fields_ = [("in_dim", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32), ("out_dim", C.c_int32),
                ("act", C.c_int32), ("out_act", C.c_int32), ("out_scale", C.c_double), ("params", C.c_void_p)]


_lib = None

# every entry point of include/cbic.h with its ctypes signature
_SIGS = {
    "cbic_last_error": (C.c_char_p, []),
    "cbic_version": (C.c_int32, []),
    "cbic_opts_default": (C.c_int32, [C.c_void_p]),
    "cbic_context_create": (C.c_int32, [C.c_int, C.c_size_t, C.c_void_p]),
    "cbic_context_destroy": (C.c_int32, [C.c_void_p]),
    "cbic_system_create": (C.c_int32, [C.c_void_p, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p]),
    "cbic_system_dims": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_system_destroy": (C.c_int32, [C.c_void_p]),
    "cbic_workspace_size": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "cbic_solve_batch": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_solve_batch_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_phase_times": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "cbic_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_calibrate_max_iter": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                            C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_mlp_param_count": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "cbic_mlp_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_bic_select": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                    C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "cbic_actor_rollout": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_server_opts_default": (C.c_int32, [C.c_void_p]),
    "cbic_server_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "cbic_server_submit": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]),
    "cbic_server_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_void_p]),
    "cbic_server_clock": (C.c_double, [C.c_void_p]),
    "cbic_server_get_stats": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "cbic_server_drain": (C.c_int32, [C.c_void_p]),
    "cbic_server_destroy": (C.c_int32, [C.c_void_p]),
}


def lib():
    """Load libcbic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_19699_amd.build`")
        # torch ships its own HIP runtime; load it first so that the library and
        # torch share one runtime in this process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code < 0:
        raise CbicError(code, lib().cbic_last_error().decode())
    return code


@dataclass
class Options:
    max_iter: int = 50
    psd_eps: float = 1e-6
    ls_max_trials: int = 16
    ls_beta: float = 0.5
    stop_mode: int = 0
    rtol: float = 1e-10
    lookahead_K: int = 0
    precision: int = FP64
    schedule: int = SCHED_AUTO
    iters_per_launch: int = 0
    group_lanes: int = 0
    flags: int = 0
    regularization: int = REG_CLIP
    lm_mu0: float = 1e-6
    lm_factor: float = 10.0
    lm_mu_max: float = 1e10
    u_max: float = float("inf")  # control bound |u_k,i| <= u_max of eq. 1; inf: none
    wg_per_cu: int = 0  # workgroup schedule: instances per compute unit (1, 2; 0 automatic)

    def c(self) -> _Opts:
        o = _Opts()
        _check(lib().cbic_opts_default(C.byref(o)))
        for f in ("max_iter", "psd_eps", "ls_max_trials", "ls_beta", "stop_mode", "rtol", "lookahead_K",
                  "precision", "schedule", "iters_per_launch", "group_lanes", "flags", "regularization",
                  "lm_mu0", "lm_factor", "lm_mu_max", "u_max", "wg_per_cu"):
            setattr(o, f, getattr(self, f))
        return o


class Context:
    def __init__(self, device: int = 0, workspace_cap: int = 0):
        self.h = C.c_void_p()
        _check(lib().cbic_context_create(device, workspace_cap, C.byref(self.h)))
        self.device = device

    def phase_times(self):
        """(init, iterations, finalisation) milliseconds of the last timed solve."""
        ms = (C.c_double * 3)()
        _check(lib().cbic_phase_times(self.h, ms))
        return tuple(ms)

    def close(self):
        if self.h:
            _check(lib().cbic_context_destroy(self.h))
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class System:
    def __init__(self, ctx: Context | None, kind: int, params):
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.kind = kind
        self.ctx = ctx
        self.h = C.c_void_p()
        _check(lib().cbic_system_create(ctx.h if ctx else None, kind, self.params.ctypes.data,
                                        self.params.size, C.byref(self.h)))
        n, m = C.c_int32(), C.c_int32()
        _check(lib().cbic_system_dims(self.h, C.byref(n), C.byref(m)))
        self.n, self.m = n.value, m.value

    def workspace_size(self, B, T_max, opts: Options | None = None):
        o = (opts or Options()).c()
        v = C.c_size_t()
        _check(lib().cbic_workspace_size(self.h, B, T_max, C.byref(o), C.byref(v)))
        return v.value

    def close(self):
        if self.h:
            _check(lib().cbic_system_destroy(self.h))
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Outputs:
    """Device tensors of one solve (torch, on the context's GPU)."""
    X: object
    U: object
    J: object
    iters: object
    status: object
    Vbar: object = None
    Vx: object = None
    xK: object = None
    cost_trace: object = None
    work: object = None
    jtrace: object = None

    @staticmethod
    def allocate(B, T_max, n, m, device, targets=True, trace_iters=None, work=True):
        import torch
        f64 = dict(dtype=torch.float64, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        return Outputs(
            X=torch.empty(B, T_max + 1, n, **f64), U=torch.empty(B, T_max, m, **f64),
            J=torch.empty(B, **f64), iters=torch.empty(B, **i32), status=torch.empty(B, **i32),
            Vbar=torch.empty(B, T_max + 1, **f64) if targets else None,
            Vx=torch.empty(B, T_max + 1, n, **f64) if targets else None,
            xK=torch.empty(B, T_max + 1, n, **f64) if targets else None,
            cost_trace=torch.empty(B, trace_iters + 1, **f64) if trace_iters is not None else None,
            work=torch.empty(B, 4, **i32) if work else None,
            jtrace=torch.empty(B, max(trace_iters, 1), **i32) if trace_iters is not None else None)

    def c(self) -> _Outputs:
        o = _Outputs()
        for f in _Outputs._fields_:
            t = getattr(self, f[0])
            setattr(o, f[0], None if t is None else t.data_ptr())
        return o


def _dptr(t):
    return None if t is None else t.data_ptr()


def solve_batch(ctx: Context, sys: System, x0, T_max: int, T=None, U0=None, opts: Options | None = None,
                out: Outputs | None = None, targets=True, trace=False, stream=None) -> Outputs:
    """Enqueue a batched solve; inputs are torch device tensors (float64 / int32)."""
    import torch
    opts = opts or Options()
    dev = torch.device("cuda", ctx.device)
    x0 = x0.to(device=dev, dtype=torch.float64).contiguous()
    B = x0.shape[0]
    if T is not None:
        T = T.to(device=dev, dtype=torch.int32).contiguous()
    if U0 is not None:
        U0 = U0.to(device=dev, dtype=torch.float64).contiguous()
    if out is None:
        out = Outputs.allocate(B, T_max, sys.n, sys.m, dev, targets=targets,
                               trace_iters=opts.max_iter if trace else None)
    o = opts.c()
    oc = out.c()
    st = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    _check(lib().cbic_solve_batch(ctx.h, sys.h, B, T_max, _dptr(T), x0.data_ptr(), _dptr(U0), C.byref(o),
                                  C.byref(oc), st))
    out._keep = (x0, T, U0)  # keep inputs alive until the caller synchronises
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def solve_batch_noalloc(ctx: Context, sys: System, x0, T_max: int, out: Outputs, T=None, U0=None,
                        opts: Options | None = None, stream=None) -> Outputs:
    """Enqueue a solve through the allocation-free entry point: the caller
    provides every device buffer (inputs as float64 / int32 device tensors,
    `out` from Outputs.allocate); the library's fixed device scratch is the
    workspace."""
    import torch
    opts = opts or Options()
    o = opts.c()
    oc = out.c()
    st = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", ctx.device)).cuda_stream
    _check(lib().cbic_solve_batch_noalloc(ctx.h, sys.h, x0.shape[0], T_max, _dptr(T), x0.data_ptr(), _dptr(U0),
                                          C.byref(o), C.byref(oc), st))
    return out


def autotune(ctx: Context, sys: System, x0, T_max: int, T=None, U0=None, opts: Options | None = None,
             stream=None):
    """Time every schedule candidate on this problem (lanes per instance, or
    the workgroup schedule's instances per compute unit); the context keeps
    the fastest for later solves that leave the choice at 0.  Returns
    (choice, ms)."""
    import torch
    opts = opts or Options()
    dev = torch.device("cuda", ctx.device)
    x0 = x0.to(device=dev, dtype=torch.float64).contiguous()
    T = None if T is None else T.to(device=dev, dtype=torch.int32).contiguous()
    U0 = None if U0 is None else U0.to(device=dev, dtype=torch.float64).contiguous()
    o = opts.c()
    g, ms = C.c_int32(), C.c_double()
    st = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    _check(lib().cbic_autotune(ctx.h, sys.h, x0.shape[0], T_max, _dptr(T), x0.data_ptr(), _dptr(U0), C.byref(o),
                               st, C.byref(g), C.byref(ms)))
    return g.value, ms.value


def calibrate_max_iter(ctx: Context, sys: System, x0, T_max: int, T=None, opts: Options | None = None,
                       cap: int = 1000, stream=None):
    """Iteration budget from a tolerance-stop solve of this batch (paper Sec.
    IV-A): returns (p99, p50, hist), the nearest-rank 99th and 50th
    percentiles of the per-instance iteration counts and their histogram
    (cap + 1 entries)."""
    import numpy as np
    import torch
    opts = opts or Options()
    dev = torch.device("cuda", ctx.device)
    x0 = x0.to(device=dev, dtype=torch.float64).contiguous()
    T = None if T is None else T.to(device=dev, dtype=torch.int32).contiguous()
    o = opts.c()
    p99, p50 = C.c_int32(), C.c_int32()
    hist = np.zeros(cap + 1, dtype=np.int64)
    st = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
    _check(lib().cbic_calibrate_max_iter(ctx.h, sys.h, x0.shape[0], T_max, _dptr(T), x0.data_ptr(), C.byref(o),
                                         cap, st, C.byref(p99), C.byref(p50),
                                         hist.ctypes.data_as(C.c_void_p)))
    return p99.value, p50.value, hist


# ---------------------------------------------------------------- networks
ACT_TANH, ACT_ELU, ACT_RELU = 0, 1, 2
OUT_LINEAR, OUT_TANH, OUT_SOFTPLUS = 0, 1, 2


@dataclass
class Mlp:
    """A perceptron for the biased initial-state selection and the actor warm
    start: `params` is a float32 device tensor in the library's packed layout
    (see cbic_mlp in include/cbic.h)."""
    in_dim: int
    width: int
    depth: int
    out_dim: int
    params: object  # torch.Tensor, float32, on the device
    act: int = ACT_TANH
    out_act: int = OUT_LINEAR
    out_scale: float = 1.0

    def c(self) -> _Mlp:
        import torch
        if self.params.dtype != torch.float32 or not self.params.is_contiguous() or not self.params.is_cuda:
            raise ValueError("network parameters must be a contiguous float32 device tensor")
        m = _Mlp(self.in_dim, self.width, self.depth, self.out_dim, self.act, self.out_act, self.out_scale,
                 self.params.data_ptr())
        n = C.c_int64()
        _check(lib().cbic_mlp_param_count(C.byref(m), C.byref(n)))
        if self.params.numel() < n.value:
            raise ValueError(f"the network needs {n.value} parameters, the tensor holds {self.params.numel()}")
        return m

    def param_count(self) -> int:
        n = C.c_int64()
        m = _Mlp(self.in_dim, self.width, self.depth, self.out_dim, self.act, self.out_act, self.out_scale, None)
        _check(lib().cbic_mlp_param_count(C.byref(m), C.byref(n)))
        return n.value


def _stream(ctx, stream):
    import torch
    return stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", ctx.device)).cuda_stream


def mlp_forward(ctx: Context, net: Mlp, x, stream=None):
    """net(x) for float32 device rows x [B][in_dim]."""
    import torch
    x = x.to(dtype=torch.float32).contiguous()
    y = torch.empty((x.shape[0], net.out_dim), dtype=torch.float32, device=x.device)
    m = net.c()
    _check(lib().cbic_mlp_forward(ctx.h, C.byref(m), x.shape[0], x.data_ptr(), y.data_ptr(), _stream(ctx, stream)))
    return y


def bic_select(ctx: Context, std_critic: Mlp, x, T, T_max: int, N: int, gather=False, stream=None):
    """Biased initial-state selection (paper Sec. III-D): returns (scores, sel),
    the std-critic's score of each candidate (x_i, tau_i = (T_max - T_i) / T_max)
    and the indices of the N highest scores in ascending order; with gather=True
    also the selected states [N][n] and horizons [N] (the next TO batch).
    x [Bc][n] and T [Bc] (or None: the network takes the state alone) are
    device tensors."""
    import torch
    x = x.to(dtype=torch.float64).contiguous()
    T = None if T is None else T.to(device=x.device, dtype=torch.int32).contiguous()
    Bc, n = x.shape
    score = torch.empty(Bc, dtype=torch.float32, device=x.device)
    sel = torch.empty(N, dtype=torch.int32, device=x.device)
    xs = torch.empty((N, n), dtype=torch.float64, device=x.device) if gather else None
    Ts = torch.empty(N, dtype=torch.int32, device=x.device) if gather and T is not None else None
    m = std_critic.c()
    _check(lib().cbic_bic_select(ctx.h, C.byref(m), Bc, n, x.data_ptr(), _dptr(T), T_max, N, score.data_ptr(),
                                 sel.data_ptr() if N > 0 else None, _dptr(xs) if N > 0 else None,
                                 _dptr(Ts) if N > 0 else None, _stream(ctx, stream)))
    return (score, sel, xs, Ts) if gather else (score, sel)


def actor_rollout(ctx: Context, sys: System, actor: Mlp, x0, T_max: int, T=None, states=False, stream=None):
    """Actor warm start (paper Sec. II): U [B][T_max][m] (and X [B][T_max+1][n]
    with states=True) of the rollouts u_k = actor(x_k, tau_k) from x0."""
    import torch
    x0 = x0.to(dtype=torch.float64).contiguous()
    B = x0.shape[0]
    T = None if T is None else T.to(device=x0.device, dtype=torch.int32).contiguous()
    U = torch.empty((B, T_max, sys.m), dtype=torch.float64, device=x0.device)
    X = torch.empty((B, T_max + 1, sys.n), dtype=torch.float64, device=x0.device) if states else None
    m = actor.c()
    _check(lib().cbic_actor_rollout(ctx.h, sys.h, C.byref(m), B, T_max, _dptr(T), x0.data_ptr(), U.data_ptr(),
                                    _dptr(X), _stream(ctx, stream)))
    return (U, X) if states else U


# ---------------------------------------------------------------- serving
class Server:
    def __init__(self, ctx: Context, mem_cap=32 << 30, slots_per_class=4096, t_max=200, iters_per_launch=4):
        o = _ServerOpts()
        _check(lib().cbic_server_opts_default(C.byref(o)))
        o.mem_cap_bytes = mem_cap
        o.slots_per_class = slots_per_class
        o.t_max = t_max
        o.iters_per_launch = iters_per_launch
        self.h = C.c_void_p()
        _check(lib().cbic_server_create(ctx.h, C.byref(o), C.byref(self.h)))
        self.ctx = ctx
        self._req = {}

    def submit(self, sys: System, x0, T: int, U0=None, opts: Options | None = None) -> int:
        x0 = np.ascontiguousarray(x0, dtype=np.float64)
        U0c = None if U0 is None else np.ascontiguousarray(U0, dtype=np.float64)
        o = (opts or Options()).c()
        tk = C.c_uint64()
        _check(lib().cbic_server_submit(self.h, sys.h, T, x0.ctypes.data,
                                        None if U0c is None else U0c.ctypes.data, C.byref(o), C.byref(tk)))
        self._req[tk.value] = (sys.n, sys.m, T)
        return tk.value

    def poll(self, ticket: int, targets=True):
        n, m, T = self._req[ticket]
        X = np.zeros((T + 1, n))
        U = np.zeros((T, m))
        Vb = np.zeros(T + 1) if targets else None
        Vx = np.zeros((T + 1, n)) if targets else None
        r = _Result()
        r.X, r.U = X.ctypes.data, U.ctypes.data
        r.Vbar = None if Vb is None else Vb.ctypes.data
        r.Vx = None if Vx is None else Vx.ctypes.data
        code = _check(lib().cbic_server_poll(self.h, ticket, C.byref(r)))
        if code == NOT_READY:
            return None
        del self._req[ticket]
        return dict(X=X, U=U, Vbar=Vb, Vx=Vx, J=r.J, iters=r.iters, status=r.status,
                    t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done)

    def clock(self) -> float:
        return lib().cbic_server_clock(self.h)

    def stats(self) -> dict:
        st = _ServerStats()
        _check(lib().cbic_server_get_stats(self.h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def drain(self):
        _check(lib().cbic_server_drain(self.h))

    def close(self):
        if self.h:
            _check(lib().cbic_server_destroy(self.h))
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
