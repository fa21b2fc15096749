"""Benchmark: converged TO solves per second on one MI355X.

Headline workload (one "step"): one batched solve of the 2-D point-mass OCP with
16384 initial states, horizon 100, dt 0.01, three soft obstacles (seeded),
through the C ABI, inputs already resident in device memory.  Forms timed:
plain FP64 with the fixed 50-iteration budget, plain FP64 with the
relative-decrease stop, and the mixed FP32/FP64 form with the
relative-decrease stop at 1e-7 (its rounding floor) and at 1e-4 (the accuracy
the metric asks for: iLQR converges quadratically, so a step that lowers J by
less than 1e-4 leaves a gap far below it).  A solve counts as converged when
its cost is within 1e-4 relative of the plain FP64 fixed-budget GPU solve of
the same instance; `value` is the converged solves per second of the fastest
form (instances outside the bar do not count).  A form's `ms_per_step` is the
wall-clock time of K solves between two device synchronisations, with two
batches in flight (--in-flight: each on a context and stream of its own, so
one batch's tail overlaps the next one's start; every batch is a whole solve);
`serial` gives the same K solves one at a time on one stream, and the p50/p99
latencies come from a further pass of K solves, each between a pair of stream
events.

The same run measures the other workloads (64 point-mass instances for
latency, 4096 arm instances with horizons 50..200, 1024 quadruped-sized
instances) and the serving loop, each with the roofline of its dominant
kernel (HIP events around the iteration kernel on its stream, which for a
lane-schedule solve also finalises the instances; algorithmic bytes or flops
from the per-instance work counters and the output sizes) and the FP64 CPU
oracle timed on a bounded sample on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "converged TO solves/sec at 1e-4 rel cost vs FP64 plain; p50/p99 latency"
SERVING_RATES = (1000, 2000, 5000, 10000, 20000, 50000)


# HBM traffic of the dominant kernels from rocprofv3 counter runs (FETCH_SIZE,
# then WRITE_SIZE, KiB per dispatch, each in a run of its own), scaled by what
# the same counters read for a plain 512 MiB device copy: FETCH_SIZE read
# 262159 KiB and WRITE_SIZE 524288 KiB for 524288 KiB moved each way.  An
# entry holds only while the sources it was taken from are unchanged (their
# sha256 is recorded); otherwise traffic is reported as null.
FETCH_SCALE = 524288.0 / 262159.0
WRITE_SCALE = 524288.0 / 524288.0
# (the kernels' sources, and the host code that orders the slots they iterate)
LANE_SOURCES = ("dev_common.hpp", "dev_systems.hpp", "ilqr_lane.hpp", "lane_launch.hpp", "runtime.hpp",
                "common.hip", "capi.cpp")
QUAD_SOURCES = ("dev_common.hpp", "ilqr_lane.hpp", "lane_launch.hpp", "runtime.hpp", "k_group_quad.hip",
                "common.hip", "capi.cpp")
# per launch, from the counter runs listed in each profile (sq_active_inst_valu:
# SQ_ACTIVE_INST_VALU, in 4-cycle units)
COUNTERS = {
    ("pm16k", "mixed_tol1e-4", "lane_iterate<PointMass,float,8,false,true>"): {
        "sources": LANE_SOURCES + ("k_lane_pm.hip",),
        "sha256": "9c945d2073fde3f7d4f5a917d77d086e48843cb29ecd4b04ff0c66a193d4d5bc",
        "fetch_kib": 265724.1, "write_kib": 494885.6, "sq_active_inst_valu": 175081598.3,
        "profile": "profiles/lane_iterate_pointmass_16k_mixed_tol.md",
    },
    ("arm4k", "mixed_tol1e-7", "lane_iterate<Arm3,float,16,false,true>"): {
        "sources": LANE_SOURCES + ("k_lane_arm.hip",),
        "sha256": "28f1166092157891156f1f68a86fd118fa463c17c93c8ad20c3502f54f36b82f",
        "fetch_kib": 1491516.9, "write_kib": 12274332.1, "sq_active_inst_valu": 5090266665.3,
        "profile": "profiles/lane_iterate_arm3_4k_mixed_tol.md",
    },
    ("quad1k", "mixed_tol1e-4", "quad_iterate<float,false,false,2>"): {
        "sources": QUAD_SOURCES,
        "sha256": "9a81d630ae82dc350a898962b5ef1ceced463dc8bbb150f32f33a08f5d77680c",
        "fetch_kib": 1939390.4, "write_kib": 2120827.7, "sq_active_inst_valu": 2292687872.0,
        "profile": "profiles/quad_iterate_1k_mixed_tol.md",
    },
}


def sources_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2602_19699_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _counters(name, form, kernel):
    e = COUNTERS.get((name, form, kernel))
    if e is None or e["sha256"] != sources_sha(e["sources"]):
        return None
    return e


def traffic_for(name, form, kernel):
    e = _counters(name, form, kernel)
    if e is None:
        return None
    return round((e["fetch_kib"] * FETCH_SCALE + e["write_kib"] * WRITE_SCALE) * 1024.0)


# VALU issue capacity: a wave64 VALU instruction occupies its SIMD's 16 lanes
# for 4 cycles (FP32 without packing, and FP64), so the chip issues at most
# 1024 SIMDs x 2.4e9 / 4 wave instructions per second.  SQ_ACTIVE_INST_VALU
# counts the issued wave instructions in those 4-cycle units (it agrees with
# SQ_INSTS_VALU within 5 %).
N_SIMD, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4


def valu_issue_frac(name, form, kernel, iterate_ms):
    """Fraction of the chip's VALU issue capacity the kernel used, from the
    SQ_ACTIVE_INST_VALU count per launch of a counter run of the same sources
    and the kernel's duration measured live."""
    e = _counters(name, form, kernel)
    if e is None or "sq_active_inst_valu" not in e:
        return None
    return e["sq_active_inst_valu"] * VALU_CYCLES / (N_SIMD * CLOCK_HZ * iterate_ms * 1e-3)


def riccati_flops(n, m):
    """Dense, symmetry-unaware flop count of one backward Riccati step."""
    return 4 * n ** 3 + 6 * n * n * m + 2 * m * m * n + 2 * m * m * (n + 1) + m ** 3 / 3 + 2 * n * n + 4 * n * m


def alg_bytes(work, Tb, n, m, elem):
    """Algorithmic HBM bytes of the iteration kernel from the instances' work
    counters: a backward sweep reads x_T and, per step, x_k, u_k and writes
    K_k (m x n), k_k (m); a line-search rollout step reads x_k, u_k, K_k, k_k
    and, when it writes, stores x_{k+1} and u_k."""
    work = work.astype(np.float64)
    sweeps, reads, writes = work[:, 0], work[:, 2], work[:, 3]
    per_step = n + m + m * n + m
    words = sweeps * (Tb * per_step + n) + reads * per_step + writes * (n + m)
    return float(words.sum() * elem)


def final_bytes(Tb, Tmax, n, m, elem, targets=True):
    """Algorithmic HBM bytes of the finalisation, which a solve in one launch
    runs inside the iteration kernel: it reads each instance's final
    trajectory (x_0..x_T, u_0..u_{T-1}) and writes the FP64 outputs padded to
    T_max (X, U and, with the critic targets, V-bar, V_x and x_{k+K}) and the
    per-instance scalars (J, iterations, status, the four work counters)."""
    Tb = np.asarray(Tb, np.float64)
    reads = ((Tb + 1) * n + Tb * m).sum() * elem
    rows = (Tmax + 1) * n + Tmax * m + ((Tmax + 1) * (1 + 2 * n) if targets else 0)
    writes = len(Tb) * (rows * 8 + 32)
    return float(reads + writes)


def alg_flops(work, Tb, n, m):
    """Algorithmic flops of the backward sweeps (dense Riccati count per step)."""
    return float((work[:, 0].astype(np.float64) * Tb).sum() * riccati_flops(n, m))


# batches in flight in the throughput loop (set from --in-flight)
IN_FLIGHT = 2


def time_form(ctx, sysm, x0d, T, Td, opts, steps, warmup, autotune=True):
    """Time one form.  Throughput: `steps` batches with IN_FLIGHT of them in
    flight, on as many contexts (each with its own workspace) and streams,
    taking the batches in turn; every batch is the whole solve.  Also the same
    steps one at a time on one context, the per-batch latency from a pass with
    stream events around every solve, and the phase times of one solve."""
    import torch
    from paper_2602_19699_amd import cbic
    dev = x0d.device
    B = x0d.shape[0]
    out = cbic.Outputs.allocate(B, T, sysm.n, sysm.m, dev, targets=True)
    width = None
    if autotune:  # lanes per instance, or the quadruped's workgroups per CU
        width, _ = cbic.autotune(ctx, sysm, x0d, T, T=Td, opts=opts)
    for _ in range(warmup):
        cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=opts, out=out)
    torch.cuda.synchronize(dev)
    stream = torch.cuda.current_stream(dev)
    # throughput with batches in flight: context 0 and IN_FLIGHT - 1 more, the
    # schedule the autotuner chose passed explicitly
    nf = max(1, IN_FLIGHT)
    popts = opts if width is None else cbic.Options(
        **{**opts.__dict__, ("wg_per_cu" if sysm.kind == 3 else "group_lanes"): width})
    ctxs = [ctx] + [cbic.Context(ctx.device) for _ in range(nf - 1)]
    syss = [sysm] + [cbic.System(c, sysm.kind, sysm.params) for c in ctxs[1:]]
    outs = [out] + [cbic.Outputs.allocate(B, T, sysm.n, sysm.m, dev, targets=True) for _ in ctxs[1:]]
    strs = [torch.cuda.Stream(dev) for _ in ctxs]
    try:
        for _ in range(max(1, warmup)):
            for c, sy, o, st in zip(ctxs, syss, outs, strs):
                cbic.solve_batch(c, sy, x0d, T, T=Td, opts=popts, out=o, stream=st.cuda_stream)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for k in range(steps):
            i = k % nf
            cbic.solve_batch(ctxs[i], syss[i], x0d, T, T=Td, opts=popts, out=outs[i], stream=strs[i].cuda_stream)
        torch.cuda.synchronize(dev)
        wall = (time.perf_counter() - t0) / steps
        # every context's last batch gave the same bits
        same = all(bool(torch.equal(o.J, outs[0].J)) and bool(torch.equal(o.U, outs[0].U)) for o in outs[1:])
    finally:
        for sy in syss[1:]:
            sy.close()
        for c in ctxs[1:]:
            c.close()
    # the same steps one at a time: back to back on one context and stream
    t0 = time.perf_counter()
    for _ in range(steps):
        cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=opts, out=out)
    torch.cuda.synchronize(dev)
    serial = (time.perf_counter() - t0) / steps
    # per-batch latency: the same number of steps again, each between a pair
    # of stream events (the events' own cost stays out of the throughput)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=opts, out=out)
        e1.record(stream)
    torch.cuda.synchronize(dev)
    lat = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
    topts = cbic.Options(**{**opts.__dict__, "flags": opts.flags | cbic.FLAG_TIMING})
    cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=topts, out=out)
    ph = ctx.phase_times()
    torch.cuda.synchronize(dev)
    return out, wall * 1e3, lat, ph, width, serial * 1e3, same


def workload_bench(ctx, name, forms, steps, warmup, cpu_sample, cpu_opts_form, quick=False):
    import torch
    from paper_2602_19699_amd import cbic, inputs as I
    dev = torch.device("cuda", 0)
    kind, params, x0, T, Tb = I.workload(name)
    B = len(x0)
    sysm = cbic.System(ctx, kind, params)
    x0d = torch.as_tensor(x0, device=dev)
    Td = None if Tb is None else torch.as_tensor(Tb, device=dev)
    Tvec = np.full(B, T) if Tb is None else Tb.astype(np.int64)
    ref = cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=cbic.Options(max_iter=50), targets=False)
    torch.cuda.synchronize(dev)
    Jref = ref.J.cpu().numpy()
    n, m = sysm.n, sysm.m
    # iteration budget (paper Sec. IV-A): the 99th percentile of a
    # tolerance-stop solve's iteration counts under a cap of 1000, then the
    # fixed-budget FP64 solve at that budget timed as a form of its own
    calib = None
    if "fp64_fixed50" in forms:
        t0 = time.perf_counter()
        p99, p50, hist = cbic.calibrate_max_iter(ctx, sysm, x0d, T, T=Td, opts=cbic.Options(rtol=1e-10), cap=1000)
        calib = {"cap": 1000, "rtol": 1e-10, "p99": p99, "p50": p50, "max": int(np.nonzero(hist)[0].max()),
                 "frac_at_cap": float(hist[1000] / hist.sum()), "seconds": round(time.perf_counter() - t0, 3)}
        if p99 < 1000:  # a budget at the cap would only time the cap
            forms = {**forms, "fp64_fixed_p99": cbic.Options(max_iter=p99)}
    results = {}
    Jforms = {}
    bounded_ref = {}  # u_max -> J of the FP64 50-iteration solve under that bound
    for fname, opts in forms.items():
        out, ms, lat, ph, width, serial_ms, same = time_form(ctx, sysm, x0d, T, Td, opts, steps, warmup)
        J = out.J.cpu().numpy()
        Jforms[fname] = J
        work = out.work.cpu().numpy()
        Jr = Jref
        if np.isfinite(opts.u_max):
            # a bounded form solves another problem: its reference is the FP64
            # solve under the same bound
            if opts.u_max not in bounded_ref:
                rb = cbic.solve_batch(ctx, sysm, x0d, T, T=Td, opts=cbic.Options(max_iter=50, u_max=opts.u_max),
                                      targets=False)
                bounded_ref[opts.u_max] = rb.J.cpu().numpy()
            Jr = bounded_ref[opts.u_max]
        rel = np.abs(J - Jr) / np.abs(Jr)
        conv = int(np.sum(rel <= 1e-4))
        elem = 8 if opts.precision == cbic.FP64 else 4
        nb = alg_bytes(work, Tvec, n, m, elem)
        # a lane-schedule solve in one launch finalises inside the iteration
        # kernel, whose time then holds both (its finalisation phase is 0)
        fused = kind != I.SYS_QUAD_SYNTH and not (opts.flags & cbic.FLAG_GRAPH) and (
            opts.iters_per_launch <= 0 or opts.iters_per_launch >= opts.max_iter)
        nfin = final_bytes(Tvec, T, n, m, 8) if fused else 0.0
        nb += nfin
        nf = alg_flops(work, Tvec, n, m)
        results[fname] = dict(
            ms_per_step=ms, p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
            converged=conv, converged_frac=conv / B, solves_per_s=B / (ms / 1e3),
            converged_solves_per_s=conv / (ms / 1e3), max_rel_cost_vs_fp64=float(np.nanmax(rel)),
            iterate_ms=ph[1], init_ms=ph[0], final_ms=ph[2], iterate_alg_bytes=nb,
            iterate_includes_finalize=fused, finalize_alg_bytes=nfin,
            iterate_GBps=nb / (ph[1] / 1e3) / 1e9, iterate_alg_flops=nf,
            iterate_TFLOPs=nf / (ph[1] / 1e3) / 1e12, mean_iters=float(out.iters.float().mean().item()),
            mean_sweeps=float(work[:, 0].mean()), batches_in_flight=IN_FLIGHT, in_flight_outputs_identical=same,
            serial_ms_per_step=serial_ms, serial_converged_solves_per_s=conv / (serial_ms / 1e3))
        results[fname]["wg_per_cu" if sysm.kind == 3 else "lanes_per_instance"] = width
        if np.isfinite(opts.u_max):
            Uo = out.U.cpu().numpy()
            results[fname]["u_max"] = opts.u_max
            results[fname]["frac_instances_at_bound"] = float(np.mean(np.any(np.abs(Uo) >= opts.u_max, axis=(1, 2))))
            results[fname]["max_abs_u"] = float(np.abs(Uo).max())
    # forms ending in "_lm" are the Levenberg-Marquardt ablation (Sec. IV-B),
    # reported beside their clipped counterpart; forms with "_umax" solve the
    # problem with the control bound of eq. 1; neither is the headline form
    best = max((k for k in results if not k.endswith("_lm") and "_umax" not in k),
               key=lambda k: results[k]["converged_solves_per_s"])
    if Tb is not None:
        # lockstep efficiency of a ragged batch: the horizon sort puts 64 / GL
        # instances of similar horizon in a wave, and a wave steps as long as
        # its longest; useful steps / stepped lane-steps for the best form
        gl = results[best]["lanes_per_instance"] or 1
        per = max(1, 64 // gl)
        srt = np.sort(Tb.astype(np.int64))[::-1]
        stepped = sum(int(srt[i]) * min(per, len(srt) - i) for i in range(0, len(srt), per))
        for r in results.values():
            r["lockstep_efficiency"] = float(srt.sum() / stepped)
    for fname in [k for k in results if k.endswith("_lm")]:
        base = fname[:-3]
        if base in results:
            a, b = results[base], results[fname]
            d = (Jforms[fname] - Jforms[base]) / np.abs(Jforms[base])
            b["vs_clip"] = {
                "clip_form": base, "time_ratio": b["ms_per_step"] / a["ms_per_step"],
                "iterate_time_ratio": b["iterate_ms"] / a["iterate_ms"],
                "mean_iters": [a["mean_iters"], b["mean_iters"]], "mean_sweeps": [a["mean_sweeps"], b["mean_sweeps"]],
                "median_rel_cost_diff": float(np.nanmedian(d)), "frac_lower_cost": float(np.mean(d < -1e-9)),
                "frac_higher_cost": float(np.mean(d > 1e-9))}
    cpu = None
    if cpu_sample and not quick:
        from oracle import oracle as orc
        ns = min(cpu_sample, B)
        threads = orc.max_threads()
        fo = forms[cpu_opts_form]
        oo = orc.Options(max_iter=fo.max_iter, stop_mode=fo.stop_mode, rtol=max(fo.rtol, 1e-10))
        t0 = time.perf_counter()
        ores = orc.solve_batch(kind, params, x0[:ns], T, T=None if Tb is None else Tb[:ns], opts=oo, nthreads=threads)
        dt = time.perf_counter() - t0
        # every form's cost against the FP64 oracle on the sampled instances
        Jo = np.asarray(ores.J)
        for fname, J in Jforms.items():
            if np.isfinite(forms[fname].u_max):
                continue  # the oracle leg solves the unbounded problem
            r = np.abs(J[:ns] - Jo) / np.abs(Jo)
            results[fname]["vs_oracle"] = {
                "oracle_form": cpu_opts_form, "instances": int(ns), "max_rel_cost": float(np.nanmax(r)),
                "median_rel_cost": float(np.nanmedian(r)), "frac_within_1e-9": float(np.mean(r <= 1e-9)),
                "frac_within_1e-4": float(np.mean(r <= 1e-4))}
        cpu = {"value": round(ns / dt, 2), "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"{'all' if ns == B else 'first %d of the' % ns} {B} instances, FP64, "
                         f"{'tolerance stop rtol=%g' % oo.rtol if oo.stop_mode else 'fixed %d iterations' % oo.max_iter}"
                         f", {threads} OpenMP threads, {dt:.2f} s"}
        # the same oracle on one core, on an eighth of that sample
        n1 = max(1, ns // 8)
        t0 = time.perf_counter()
        orc.solve_batch(kind, params, x0[:n1], T, T=None if Tb is None else Tb[:n1], opts=oo, nthreads=1)
        d1 = time.perf_counter() - t0
        cpu["single_core"] = {"value": round(n1 / d1, 2), "unit": "solves/s", "sample": f"first {n1} instances, "
                              f"{d1:.2f} s"}
    sysm.close()
    return results, best, cpu, calib


def roofline_for(name, form, res, form_opts):
    prec = "double" if form_opts.precision == 0 else "float"
    if name == "quad1k":
        # the Riccati products run as MFMA tiles: the dense matrix-core peak of the form's precision
        peak = FP64_PEAK_TFLOPS if form_opts.precision == 0 else FP32_PEAK_TFLOPS
        box = "true" if np.isfinite(form_opts.u_max) else "false"
        lm = "true" if form_opts.regularization == 1 else "false"
        kernel = f"quad_iterate<{prec},{box},{lm},{res['wg_per_cu']}>"
        vf = valu_issue_frac(name, form, kernel, res["iterate_ms"])
        return {"bound": "mfma", "achieved": round(res["iterate_TFLOPs"], 4), "peak": peak, "unit": "TFLOP/s",
                "frac": round(res["iterate_TFLOPs"] / peak, 5), "traffic": traffic_for(name, form, kernel),
                "kernel": kernel, "alg_flops_per_launch": res["iterate_alg_flops"],
                "iterate_ms": round(res["iterate_ms"], 4),
                "valu_issue_frac": None if vf is None else round(vf, 4)}
    sysname = {"pm16k": "PointMass", "pm64": "PointMass", "arm4k": "Arm3"}[name]
    bounded = "true" if np.isfinite(form_opts.u_max) else "false"
    fin = "true" if res.get("iterate_includes_finalize") else "false"
    kernel = f"lane_iterate<{sysname},{prec},{res['lanes_per_instance']},{bounded},{fin}>"
    vf = valu_issue_frac(name, form, kernel, res["iterate_ms"])
    return {"bound": "hbm", "achieved": round(res["iterate_GBps"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(res["iterate_GBps"] / HBM_PEAK_GBS, 5), "traffic": traffic_for(name, form, kernel),
            "kernel": kernel, "alg_bytes_per_launch": res["iterate_alg_bytes"],
            "iterate_ms": round(res["iterate_ms"], 4),
            # the binding resource: the share of the chip's VALU issue slots the kernel used
            "valu_issue_frac": None if vf is None else round(vf, 4)}


def bic_pipeline(ctx, steps, warmup):
    """One CACTO-BIC TO batch at the headline scale (paper Sec. III-D, II):
    score 10N = 163840 point-mass candidate initial states (remaining horizons
    uniform on 1..100) with the std-critic, keep the N = 16384 most uncertain,
    roll the actor out from them as the warm start and solve the batch (mixed
    form, relative-decrease stop 1e-7).  Random-weight networks (two hidden
    layers of 64 tanh units; softplus std-critic, 10 tanh actor) stand in for
    trained ones.  Each stage is timed with HIP events on the stream."""
    import torch
    from paper_2602_19699_amd import cbic, inputs as I
    dev = torch.device("cuda", 0)
    N, Bc = 16384, 163840
    kind, params, _, T_max, _ = I.workload("pm16k", B=1)
    x, T, _ = I.bic_candidates("pm16k", Bc)
    xd, Td = torch.as_tensor(x, device=dev), torch.as_tensor(T, device=dev)
    sysm = cbic.System(ctx, kind, params)
    std = cbic.Mlp(5, 64, 2, 1, torch.as_tensor(I.mlp_params(5, 64, 2, 1, seed=101), device=dev), cbic.ACT_TANH,
                   cbic.OUT_SOFTPLUS)
    actor = cbic.Mlp(5, 64, 2, 2, torch.as_tensor(I.mlp_params(5, 64, 2, 2, seed=102), device=dev), cbic.ACT_TANH,
                     cbic.OUT_TANH, 10.0)
    opts = cbic.Options(precision=cbic.MIXED, stop_mode=1, rtol=1e-7)
    out = cbic.Outputs.allocate(N, T_max, sysm.n, sysm.m, dev, targets=True)
    stream = torch.cuda.current_stream(dev)
    cbic.autotune(ctx, sysm, xd[:N].contiguous(), T_max, T=Td[:N].contiguous(), opts=opts)

    def step(ev=None):
        if ev: ev[0].record(stream)
        _, _, xs, Ts = cbic.bic_select(ctx, std, xd, Td, T_max, N, gather=True)
        if ev: ev[1].record(stream)
        U0 = cbic.actor_rollout(ctx, sysm, actor, xs, T_max, T=Ts)
        if ev: ev[2].record(stream)
        cbic.solve_batch(ctx, sysm, xs, T_max, T=Ts, U0=U0, opts=opts, out=out)
        if ev: ev[3].record(stream)
        return Ts

    for _ in range(warmup):
        step()
    torch.cuda.synchronize(dev)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for ev in evs:
        Ts = step(ev)
    torch.cuda.synchronize(dev)
    wall = (time.perf_counter() - t0) / steps * 1e3
    st = np.array([[ev[i].elapsed_time(ev[i + 1]) for i in range(3)] for ev in evs])
    med = np.median(st, axis=0)
    iters = out.iters.float().mean().item()
    # the same solve from the zero warm start, for the iteration count
    cbic.solve_batch(ctx, sysm, out.X[:, 0].contiguous(), T_max, T=Ts, opts=opts, out=out)
    torch.cuda.synchronize(dev)
    iters0 = out.iters.float().mean().item()
    sysm.close()
    flops = 2.0 * Bc * (5 * 64 + 64 + 64 * 64 + 64 + 64 + 1)
    return {"workload": "CACTO-BIC batch: 163840 point-mass candidates (T uniform 1..100) -> std-critic scores -> "
                        "top 16384 -> actor warm start -> mixed solve (tol 1e-7); random-weight 2x64 tanh networks",
            "ms_per_batch": round(wall, 4), "select_ms": round(float(med[0]), 4), "actor_ms": round(float(med[1]), 4),
            "solve_ms": round(float(med[2]), 4), "mean_iters_actor_warm_start": round(iters, 4),
            "mean_iters_zero_warm_start": round(iters0, 4), "select_scoring_flops": flops,
            "steps": steps}


SERVING_FORMS = {
    # name: (precision, relative-decrease stop)
    "fp64_tol1e-10": (0, 1e-10),
    "mixed_tol1e-7": (1, 1e-7),
}


def serving(ctx, rates, min_requests=20000, min_seconds=0.4, batched=None):
    """Open-loop Poisson serving: requests drawn 50/30/20 from the point mass,
    the arm and the quadruped, horizons uniform on 20..200, 32 GiB memory cap,
    4 iterations per launch; for each form (FP64 and the mixed form, each with
    its relative-decrease stop) and each offered rate, max(min_requests,
    rate * min_seconds) arrivals.  Beside p50/p99 per class, the server's own
    counters over each rate: iteration launches, resident requests per launch,
    and the share of wall time its worker thread was busy (the host side's
    load).  `batched` (optional) maps a form to the batched solver's per-batch
    p99 of each class, for comparison."""
    from paper_2602_19699_amd import cbic, loadgen
    out = {"workload": "Poisson arrivals, mix 50/30/20 point mass / arm / quadruped, T~U{20..200}, cap 32 GiB, "
                       "4 iterations per launch", "forms": {}}
    for fi, (fname, (prec, rtol)) in enumerate(SERVING_FORMS.items()):
        mix = loadgen.Mix(ctx, precision=prec, stop_mode=1, rtol=rtol)
        srv = cbic.Server(ctx, mem_cap=32 << 30, slots_per_class=4096, t_max=200, iters_per_launch=4)
        loadgen.run_poisson(srv, mix, rate=1000.0, n=300, seed=1)  # warm-up: pools, code objects
        rows = []
        for i, rate in enumerate(rates):
            n = int(max(min_requests, rate * min_seconds))
            s0 = srv.stats()
            t0 = time.perf_counter()
            st, _, _ = loadgen.run_poisson(srv, mix, rate=float(rate), n=n, seed=100 + 10 * fi + i)
            wall = time.perf_counter() - t0
            s1 = srv.stats()
            launches = s1["launches"] - s0["launches"]
            st["launches"] = launches
            st["slots_per_launch"] = (s1["launched_slots"] - s0["launched_slots"]) / max(launches, 1)
            st["host_busy_frac"] = (s1["host_busy_s"] - s0["host_busy_s"]) / wall
            rows.append({k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in st.items()})
            print(f"serving {fname} {rate}/s: {rows[-1]}", file=sys.stderr, flush=True)
        out["forms"][fname] = {"rates": rows, "server_stats": srv.stats(),
                               "batched_p99_ms": None if batched is None else batched.get(fname)}
        srv.close()
    return out


def fmt(d):
    return {k: (float(f"{v:.6g}") if isinstance(v, float) else fmt(v) if isinstance(v, dict) else v)
            for k, v in d.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--quick", action="store_true", help="headline workload only, no CPU baseline, no serving")
    ap.add_argument("--in-flight", type=int, default=2,
                    help="batches in flight in the throughput loop (each on its own context and stream)")
    ap.add_argument("--only", default=None, help="time only this form (for profiler runs)")
    ap.add_argument("--workload", default=None, help="time only this workload (pm16k, pm64, arm4k, quad1k)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only three plain 512 MiB device copies (to scale the HBM byte counters)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only the serving workload: Poisson rates 1k..50k/s, one JSON line")
    ap.add_argument("--bic", action="store_true", help="only the CACTO-BIC batch pipeline, one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the instances are independent and a "
              f"multi-GPU run would shard the batch with no exchange, which this program does not launch.",
              file=sys.stderr)
        sys.exit(2)
    global IN_FLIGHT
    IN_FLIGHT = max(1, args.in_flight)

    if args.copy_calib:
        import torch
        a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 3}))
        return

    from paper_2602_19699_amd import cbic

    ctx = cbic.Context(0)
    if args.serving_sweep:
        print(json.dumps(serving(ctx, rates=SERVING_RATES)))
        return
    if args.bic:
        print(json.dumps(bic_pipeline(ctx, steps=args.steps, warmup=args.warmup)))
        return

    F = cbic.Options
    forms = {
        "pm16k": {"fp64_fixed50": F(max_iter=50), "fp64_tol1e-10": F(stop_mode=1, rtol=1e-10),
                  "mixed_tol1e-7": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7),
                  "mixed_tol1e-4": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-4),
                  "fp64_tol1e-10_lm": F(stop_mode=1, rtol=1e-10, regularization=cbic.REG_LM),
                  "mixed_tol1e-7_umax10": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7, u_max=10.0)},
        "pm64": {"fp64_fixed50": F(max_iter=50), "mixed_tol1e-7": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7),
                 "mixed_tol1e-4": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-4)},
        "arm4k": {"fp64_fixed50": F(max_iter=50), "mixed_tol1e-7": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7),
                  "fp64_tol1e-10": F(stop_mode=1, rtol=1e-10),
                  "fp64_tol1e-10_lm": F(stop_mode=1, rtol=1e-10, regularization=cbic.REG_LM),
                  "mixed_tol1e-7_umax8": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7, u_max=8.0)},
        "quad1k": {"fp64_fixed50": F(max_iter=50), "fp64_tol1e-10": F(stop_mode=1, rtol=1e-10),
                   "mixed_tol1e-7": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7),
                   "mixed_tol1e-4": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-4),
                   "fp64_tol1e-10_lm": F(stop_mode=1, rtol=1e-10, regularization=cbic.REG_LM),
                   "mixed_tol1e-7_umax5": F(precision=cbic.MIXED, stop_mode=1, rtol=1e-7, u_max=5.0)},
    }
    cpu_cfg = {"pm16k": (16384, "fp64_fixed50"), "pm64": (64, "fp64_fixed50"), "arm4k": (512, "fp64_fixed50"),
               "quad1k": (64, "fp64_tol1e-10")}
    names = ["pm16k"] if args.quick else ["pm16k", "pm64", "arm4k", "quad1k"]
    if args.workload:
        names = [args.workload]
    if args.only:
        for nme in names:
            forms[nme] = {args.only: forms[nme][args.only]}
    other = {}
    head = None
    for nme in names:
        steps = args.steps if nme in ("pm16k", "pm64") else max(3, args.steps // 4)
        res, best, cpu, calib = workload_bench(ctx, nme, forms[nme], steps, args.warmup, cpu_cfg[nme][0],
                                               cpu_cfg[nme][1], quick=args.quick or bool(args.only))
        entry = {"best_form": best, "forms": {k: fmt(v) for k, v in res.items()},
                 "roofline": roofline_for(nme, best, res[best], forms[nme][best]), "cpu_baseline": cpu,
                 "max_iter_calibration": calib, "steps": steps}
        if head is None:
            head = (nme, res, best, entry)
        else:
            other[nme] = entry
    nme, res, best, entry = head
    h = res[best]
    wl = {"pm16k": "point-mass OCP (n=4, m=2), B=16384 initial states, T=100, dt=0.01, 3 soft obstacles",
          "pm64": "point-mass OCP (n=4, m=2), B=64, T=100",
          "arm4k": "planar 3-link arm (n=6, m=3), B=4096, T uniform 50..200",
          "quad1k": "quadruped-sized system (n=37, m=12), B=1024, T=100"}[nme]
    # the batched solver's per-batch p99 of each class in the serving forms
    allforms = {nme: res, **{k: v["forms"] for k, v in other.items()}}
    batched = {fname: {cls: round(allforms[w][fname]["p99_ms"], 4)
                       for cls, w in (("pm", "pm16k"), ("arm", "arm4k"), ("quad", "quad1k"))
                       if fname in allforms.get(w, {})}
               for fname in SERVING_FORMS}
    serve = None if (args.quick or args.only or args.workload) else serving(ctx, rates=SERVING_RATES,
                                                                            batched=batched)
    bic = None if (args.quick or args.only or args.workload) else bic_pipeline(ctx, steps=10, warmup=2)
    line = {
        "metric": METRIC,
        "value": round(h["converged_solves_per_s"], 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": entry["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if forms[nme][best].precision == 0 else "f32+f64",
        "data": "synthetic (seeded system parameters and initial states)",
        "config": {"workload": wl, "form": best, "p50_ms": round(h["p50_ms"], 4), "p99_ms": round(h["p99_ms"], 4),
                   "converged_frac": round(h["converged_frac"], 5), "batches_in_flight": IN_FLIGHT},
        # the same steps one batch at a time (one context, one stream)
        "serial": {"value": round(h["serial_converged_solves_per_s"], 1),
                   "ms_per_step": round(h["serial_ms_per_step"], 4)},
        "forms": entry["forms"],
        "roofline": entry["roofline"],
        "cpu_baseline": entry["cpu_baseline"],
        "max_iter_calibration": entry["max_iter_calibration"],
        "workloads": other,
        "serving": serve,
        "bic_pipeline": bic,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
