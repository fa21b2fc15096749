"""Open-loop Poisson request generator for the serving loop.

Requests are drawn 50/30/20 from the point mass, the 3-link arm and the
37-state quadruped, with horizons uniform on 20..200, and submitted at
exponentially distributed gaps whatever the server's progress (open loop).
Latency is completion time minus the scheduled arrival time.
"""
from __future__ import annotations

import numpy as np

from . import cbic, inputs as I


class Mix:
    """The three system classes of the serving workload on one context."""

    def __init__(self, ctx, sys_seed=0, precision=cbic.FP64, stop_mode=1, rtol=1e-10, max_iter=50):
        self.ctx = ctx
        pq = I.quad_params(sys_seed)
        self.params = {I.SYS_POINT_MASS: I.point_mass_params(sys_seed), I.SYS_PLANAR3: I.planar3_params(sys_seed),
                       I.SYS_QUAD_SYNTH: pq}
        self.systems = {k: cbic.System(ctx, k, p) for k, p in self.params.items()}
        self.kinds = [I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_QUAD_SYNTH]
        self.opts = cbic.Options(precision=precision, stop_mode=stop_mode, rtol=rtol, max_iter=max_iter)

    def x0(self, kind, n, seed):
        if kind == I.SYS_POINT_MASS:
            return I.point_mass_x0(n, seed)
        if kind == I.SYS_PLANAR3:
            return I.planar3_x0(n, seed)
        return I.quad_x0(n, self.params[I.SYS_QUAD_SYNTH], seed)

    def requests(self, n, seed=0, mix=(0.5, 0.3, 0.2), t_range=(20, 200)):
        rng = np.random.default_rng(seed)
        cls = rng.choice(3, n, p=mix)
        T = rng.integers(t_range[0], t_range[1] + 1, n)
        x0s = {k: self.x0(k, n, seed + 17 * (i + 1)) for i, k in enumerate(self.kinds)}
        return [(self.kinds[c], int(T[i]), x0s[self.kinds[c]][i]) for i, c in enumerate(cls)]


def run_poisson(server: cbic.Server, mix: Mix, rate: float, n: int, seed: int = 0, t_range=(20, 200)):
    """Submit n requests at Poisson rate `rate` (1/s); return latency statistics."""
    reqs = mix.requests(n, seed, t_range=t_range)
    rng = np.random.default_rng(seed + 1)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    t0 = server.clock() + 0.01
    tickets = []
    for i, (kind, T, x0) in enumerate(reqs):
        target = t0 + arrivals[i]
        while server.clock() < target:
            pass
        tickets.append(server.submit(mix.systems[kind], x0, T, opts=mix.opts))
    server.drain()
    res = [server.poll(t, targets=False) for t in tickets]
    sched = t0 + arrivals
    done = np.array([r["t_done"] for r in res])
    sub = np.array([r["t_submit"] for r in res])
    lat = done - sched
    span = done.max() - sched[0]
    kinds = np.array([k for k, _, _ in reqs])
    out = {"rate": rate, "requests": n, "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "solves_per_s": float(n / span),
           "submit_lag_p99_ms": float(np.percentile(sub - sched, 99) * 1e3)}
    for k, name in ((I.SYS_POINT_MASS, "pm"), (I.SYS_PLANAR3, "arm"), (I.SYS_QUAD_SYNTH, "quad")):
        sel = kinds == k
        if sel.any():
            out[f"p99_ms_{name}"] = float(np.percentile(lat[sel], 99) * 1e3)
    return out, res, reqs
