"""Shared helpers for the GPU parity tests: run the same seeded workload on the
HIP path (through the C ABI) and on the FP64 CPU oracle, and compare."""
from __future__ import annotations

import dataclasses

import numpy as np

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

STATUS_MASK = 31


def gpu_solve(ctx, kind, params, x0, T_max, T=None, U0=None, trace=False, **opt):
    import torch
    from paper_2602_19699_amd import cbic
    sys_ = cbic.System(ctx, kind, params)
    try:
        o = cbic.Options(**opt)
        dev = torch.device("cuda", ctx.device)
        Tt = None if T is None else torch.as_tensor(np.asarray(T, np.int32), device=dev)
        U0t = None if U0 is None else torch.as_tensor(np.asarray(U0, np.float64), device=dev)
        out = cbic.solve_batch(ctx, sys_, torch.as_tensor(np.asarray(x0, np.float64), device=dev), T_max, T=Tt,
                               U0=U0t, opts=o, trace=trace)
        torch.cuda.synchronize(dev)
        res = {k: (None if getattr(out, k) is None else getattr(out, k).cpu().numpy())
               for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx", "xK", "cost_trace", "work", "jtrace")}
        res["status"] = res["status"].astype(np.uint32)
    finally:
        sys_.close()
    return res


def oracle_opts(**opt):
    """The oracle's options for the same keyword arguments gpu_solve takes."""
    lm = opt.get("regularization", 0) == 1
    return orc.Options(max_iter=opt.get("max_iter", 50), ls_trials=opt.get("ls_max_trials", 16),
                       stop_mode=opt.get("stop_mode", 0), lookahead=opt.get("lookahead_K", 0),
                       eps=-np.inf if lm else opt.get("psd_eps", 1e-6), beta=opt.get("ls_beta", 0.5),
                       rtol=opt.get("rtol", 1e-10), reg=1 if lm else 0, mu0=opt.get("lm_mu0", 1e-6),
                       mu_factor=opt.get("lm_factor", 10.0), mu_max=opt.get("lm_mu_max", 1e10),
                       umax=opt.get("u_max", np.inf))


def rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def compare(g, r, idx=None, tol_J=1e-9, tol_traj=None, check_status=True, rtol=1e-10, label=""):
    """Element-wise comparison of a GPU result g with oracle result r (rows idx of g)."""
    idx = np.arange(len(r.J)) if idx is None else np.asarray(idx)
    Jg = g["J"][idx]
    e = rel(Jg, r.J)
    finite = np.isfinite(r.J)
    assert np.array_equal(np.isfinite(Jg), finite), f"{label}: finiteness differs"
    worst = int(np.argmax(np.where(finite, e, 0))) if finite.any() else 0
    bad = np.where(finite & (e > tol_J))[0]
    assert len(bad) == 0, (f"{label}: {len(bad)} instances beyond {tol_J:g} rel cost; worst "
                           f"#{idx[bad[0]]} rel {e[bad[0]]:.3e} J_gpu {Jg[bad[0]]!r} J_ref {r.J[bad[0]]!r} "
                           f"iters {g['iters'][idx[bad[0]]]} vs {r.iters[bad[0]]} status "
                           f"{g['status'][idx[bad[0]]]} vs {r.status[bad[0]]}")
    if check_status:
        sg = g["status"][idx] & STATUS_MASK
        # which condition ended the solve must agree per instance, except where
        # the deciding comparison was a near-tie that rounding settles either way
        ties = 0
        for i in np.flatnonzero(sg != r.status):
            assert _status_tie(r, i, int(g["iters"][idx[i]]), rtol), (
                f"{label}: #{idx[i]} status {sg[i]} vs {r.status[i]} (iters {g['iters'][idx[i]]} vs "
                f"{r.iters[i]}) without a near-tie")
            ties += 1
        if ties:
            print(f"{label}: {ties} status differences, each at a near-tie")
    return float(e[finite].max()) if finite.any() else 0.0


def _status_tie(r, i, it_gpu, rtol, tie=1e-12):
    """Whether the oracle's run i reached a decision that rounding can flip at
    an iteration where the GPU's run (it_gpu accepted iterations) and the
    oracle's part: a relative decrease within `tie` (in units of J) of the stop
    tolerance rtol, or a line search whose trial costs came within `tie` of the
    cost they were compared with."""
    lo, hi = min(it_gpu, int(r.iters[i])), max(it_gpu, int(r.iters[i]))
    tr = r.trace[i]
    for k in range(max(lo, 1), min(hi + 1, len(tr))):
        if abs((tr[k - 1] - tr[k]) - rtol * abs(tr[k - 1])) <= tie * abs(tr[k - 1]):
            return True
    return any(r.margin[i, k] <= tie for k in range(lo, min(hi + 1, r.margin.shape[1])))


def workload(name, B=None, sys_seed=0):
    return I.workload(name, B=B, sys_seed=sys_seed)


def oracle_ensemble(kind, params, x0, T_max, T=None, U0=None, opts=None, rel_step=2.0 ** -52, probe32=False):
    """The oracle's solve and two more from x0 scaled by (1 + rel_step) and
    (1 - rel_step / 2): one ulp either way for the default step, about one
    FP32 rounding for rel_step = 2^-24.  probe32 adds the oracle's FP32-storage
    probe (Options.round32: what the mixed form keeps in FP32 rounded to FP32).
    Their spread is the instance's own sensitivity to rounding."""
    r = orc.solve_batch(kind, params, x0, T_max, T=T, U0=U0, opts=opts)
    rps = []
    for f in (1 + rel_step, 1 - rel_step / 2):
        q = orc.solve_batch(kind, params, x0 * f, T_max, T=T, U0=U0, opts=opts)
        q.x0_scale = f
        rps.append(q)
    if probe32:
        q = orc.solve_batch(kind, params, x0, T_max, T=T, U0=U0, opts=dataclasses.replace(opts, round32=1))
        q.x0_scale = 1.0
        rps.append(q)
    return r, rps


def trace_sensitivity(r, rps):
    """[B][max_iter+1]: the largest relative change, over the ensemble, of the
    cost after each number of accepted iterations."""
    out = np.zeros_like(r.trace)
    for q in rps:
        out = np.maximum(out, np.abs(q.trace - r.trace) / np.maximum(np.abs(r.trace), 1e-300))
    return np.where(np.isfinite(out), out, np.inf)


def check_parity(g, kind, params, x0, T_max, T, opts, r, rps, idx=None, tol=1e-9, onset_tol=None,
                 tie_tol=1e-12, mixed=False, U0=None, label=""):
    """Per-instance parity of a GPU result g (rows idx of the batch x0, T, U0)
    with the oracle r (one row per entry of idx), whose ensemble rps
    (oracle_ensemble) measures each instance's own sensitivity to rounding.  Every instance must fall in one of three sets:

    direct    |J_gpu - J_oracle| <= tol |J_oracle|;
    replay    the GPU's accepted line-search indices (jtrace) differ from the
              oracle's first at an iteration where the oracle's trial costs came
              within tie_tol (relative) of the cost they were compared with: a
              near-tie, decided either way by rounding.  The oracle replayed
              with the GPU's indices forced must then match to tol;
    sensitive the oracle's own cost after some iteration i_c moves by more than
              onset_tol under the ensemble's perturbation (rounding is
              amplified: closed-loop rollouts through chaotic dynamics).  The
              GPU's cost trace must match the oracle's to tol before i_c and its
              accepted indices must agree there, and the result must be valid:
              every step satisfies the dynamics, X_0 = x0, J is the trajectory's
              cost, the cost trace falls strictly over the accepted iterations
              and is constant after, the indices and the status are consistent
              with it, and an instance stopped as converged or by a failed line
              search is stationary within ten times the ensemble's largest
              adjoint gradient (max norm; projected onto the box when the
              control bound is on).  Its end condition itself is not fixed by
              the problem and is not compared.

    mixed: the GPU solve ran in the mixed form, whose trajectories are FP32
    (dynamics residual and trajectory cost then to 1e-5 relative, X_0 the
    FP32 rounding of x0).  Returns the three sets' sizes (printed)."""
    idx = np.arange(len(r.J)) if idx is None else np.asarray(idx)
    onset_tol = tol / 100 if onset_tol is None else onset_tol
    mi = opts.max_iter
    Jg = g["J"][idx]
    fin = np.isfinite(r.J)
    assert np.array_equal(np.isfinite(Jg), fin), f"{label}: finiteness differs"
    e = np.where(fin, rel(Jg, r.J), 0.0)
    direct = e <= tol
    sens = trace_sensitivity(r, rps)
    jg = g["jtrace"][idx] if g.get("jtrace") is not None else None
    trg = g["cost_trace"][idx] if g.get("cost_trace") is not None else None
    assert jg is not None and trg is not None, f"{label}: the GPU solve must return cost_trace and jtrace"
    sets = {"direct": int(direct.sum()), "replay": 0, "sensitive": 0}
    rest = np.flatnonzero(~direct)
    # replay set: first differing accepted index at a near-tie
    jr = r.jtrace[:, :mi] if mi > 0 else r.jtrace[:, :0]
    cand = [i for i in rest if mi > 0 and np.any(jg[i, :mi] != jr[i])]
    replayed = set()
    if cand:
        cand = np.asarray(cand)
        Tc = None if T is None else np.asarray(T)[idx[cand]]
        U0c = None if U0 is None else np.asarray(U0)[idx[cand]]
        rr = orc.solve_batch(kind, params, x0[idx[cand]], T_max, T=Tc, U0=U0c, opts=opts,
                             force_j=jg[cand, :mi])
        for c, i in enumerate(cand):
            d = int(np.flatnonzero(jg[i, :mi] != jr[i])[0])
            tie = r.margin[i, d] <= tie_tol
            if tie and rel(Jg[i], rr.J[c]) <= tol:
                replayed.add(int(i))
                print(f"{label}: replay #{idx[i]}: first differing index at iteration {d} "
                      f"(j gpu {jg[i, d]}, oracle {jr[i, d]}, margin {r.margin[i, d]:.1e}); replay rel "
                      f"{rel(Jg[i], rr.J[c]):.1e}")
    sets["replay"] = len(replayed)
    worst_resid = 0.0
    no_ref = 0
    for i in rest:
        if int(i) in replayed:
            continue
        b = idx[i]
        over = np.flatnonzero(sens[i] > onset_tol)
        assert len(over) > 0, (f"{label}: #{b} differs by {e[i]:.3e} (J gpu {Jg[i]!r}, oracle {r.J[i]!r}, iters "
                               f"{g['iters'][b]} vs {r.iters[i]}, status {g['status'][b]} vs {r.status[i]}) but "
                               f"its own sensitivity stays <= {onset_tol:g} (max {sens[i].max():.1e})")
        ic = int(over[0])
        # prefix: the cost trace and the accepted indices before the onset
        pre = rel(trg[i, :ic], r.trace[i, :ic])
        assert np.all(pre <= tol), f"{label}: #{b} cost trace differs before its onset {ic}: {pre.max():.2e}"
        if ic >= 2:
            assert np.array_equal(jg[i, :ic - 1], jr[i, :ic - 1]), f"{label}: #{b} indices differ before {ic}"
        worst_resid = max(worst_resid, _check_valid(g, b, kind, params, x0[b], T_max,
                                                    None if T is None else int(np.asarray(T)[b]), mi, mixed,
                                                    opts.umax, label, opts.stop_mode, opts.rtol))
        # the end condition of such an instance is not fixed by the problem (an
        # oracle run from x0 (1 + 3 ulp) may end by a failed line search where
        # three others use the budget): it must be consistent (above) and, if
        # it claims a stop, stationary
        sg = int(g["status"][b]) & STATUS_MASK
        if sg & (orc.ST_CONVERGED | orc.ST_LS_FAILED):
            Tb = T_max if T is None else int(np.asarray(T)[b])
            gn = _stationarity(kind, params, x0[b], g["U"][b, :Tb], opts.umax)
            ref = np.nanmax([_stationarity(kind, params, x0[b] * getattr(q, "x0_scale", 1.0), q.U[i, :Tb], opts.umax)
                             for q in [r] + rps])
            # the mixed form's FP32 Riccati arithmetic resolves the gains 10 to 35
            # times less finely than FP32 storage alone (the oracle's probe), so
            # the gradient at which it stops is larger in proportion
            fac = 100.0 if mixed else 10.0
            # where the oracle's own runs stop no nearer to stationarity than the
            # warm start was (blown-up rollouts: the arm's cost does not see its
            # speed) there is no reference, and the instance is counted
            U0b = np.zeros_like(g["U"][b, :Tb]) if U0 is None else np.asarray(U0)[b, :Tb]
            if np.isfinite(umax := opts.umax):
                U0b = np.clip(U0b, -umax, umax)
            g0 = _stationarity(kind, params, x0[b], U0b, opts.umax)
            if np.isfinite(ref) and ref < g0:
                assert gn <= fac * ref, f"{label}: #{b} stationarity {gn:.2e} vs the oracle's {ref:.2e}"
            else:
                no_ref += 1
        sets["sensitive"] += 1
    es = e[np.asarray([i for i in rest if int(i) not in replayed], dtype=int)]
    print(f"{label}: {len(idx)} instances: direct {sets['direct']} (max rel {e[direct].max() if direct.any() else 0:.1e}),"
          f" replay {sets['replay']}, rounding-sensitive {sets['sensitive']}"
          + (f" (their GPU-oracle rel: median {np.median(es):.1e}, max {es.max():.1e}; the oracle's own "
             f"spread: median {np.median(sens[rest, -1]):.1e}; worst dynamics residual {worst_resid:.1e}; "
             f"stopped where the oracle has no stationary reference: {no_ref})"
             if len(es) else ""))
    return sets


def _stationarity(kind, params, x0b, U, umax):
    """Max norm of the adjoint gradient of J at U, projected onto the box
    |u| <= umax (a component held at a bound counts only if it points inward)."""
    gr = orc.gradient(kind, params, x0b, U)[3]
    if np.isfinite(umax):
        gr = np.where(U >= umax, np.maximum(gr, 0.0), np.where(U <= -umax, np.minimum(gr, 0.0), gr))
    return float(np.abs(gr).max())


def _check_valid(g, b, kind, params, x0b, T_max, Tb, max_iter, mixed, umax, label, stop_mode=0, rtol=0.0):
    """Validity of one returned solve, whatever the rounding did to its path."""
    Tb = T_max if Tb is None else Tb
    X, U = g["X"][b, :Tb + 1], g["U"][b, :Tb]
    d, J = orc.check_trajectory(kind, params, X, U)
    # an FP32 step of a fast-moving arm carries a few FP32 roundings of its
    # largest intermediate (Coriolis terms ~ |qdot|^2 through an inverse mass
    # matrix of norm up to ~1e2), relative to a state of ~1e2: up to ~1e-4
    rt = 1e-3 if mixed else 1e-12
    assert d <= rt, f"{label}: #{b} dynamics residual {d:.2e}"
    assert abs(J - g["J"][b]) <= (1e-5 if mixed else 1e-12) * abs(J), f"{label}: #{b} J is not the trajectory's cost"
    x0r = x0b.astype(np.float32).astype(np.float64) if mixed else x0b
    assert np.array_equal(X[0], x0r), f"{label}: #{b} X_0 != x0"
    assert np.all(np.abs(U) <= umax), f"{label}: #{b} control outside the bound"
    it = int(g["iters"][b])
    tr = g["cost_trace"][b]
    assert np.all(np.diff(tr[:it + 1]) < 0), f"{label}: #{b} accepted costs do not fall strictly"
    assert np.all(tr[it:] == g["J"][b]), f"{label}: #{b} trace after the last accepted iteration"
    jt = g["jtrace"][b]
    st = int(g["status"][b]) & STATUS_MASK
    assert np.all(jt[:it] >= 0), f"{label}: #{b} accepted iterations without an index"
    frozen = st & (orc.ST_LS_FAILED | orc.ST_CHOL_FAIL | orc.ST_NONFINITE)
    if it < max_iter:
        assert jt[it] == (-1 if frozen else -2), f"{label}: #{b} index after the last accepted iteration"
        assert np.all(jt[it + 1:max_iter] == -2), f"{label}: #{b} indices of iterations not run"
    if st & orc.ST_MAX_ITER:
        assert it == max_iter, f"{label}: #{b} MAX_ITER after {it} iterations"
    if stop_mode == 1 and it >= 1:
        # the relative-decrease stop: taken exactly at the first accepted step
        # that lowered J by at most rtol |J_old|
        small = (tr[:it] - tr[1:it + 1]) <= rtol * np.abs(tr[:it])
        assert not small[:-1].any(), f"{label}: #{b} ran on after a step that meets the stop rule"
        assert bool(small[-1]) == bool(st & orc.ST_CONVERGED), f"{label}: #{b} CONVERGED and the stop rule disagree"
    return d
