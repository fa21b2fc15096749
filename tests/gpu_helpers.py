"""Shared helpers for the GPU parity tests: run the same seeded workload on the
HIP path (through the C ABI) and on the FP64 CPU oracle, and compare."""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

STATUS_MASK = 31


def gpu_solve(ctx, kind, params, x0, T_max, T=None, U0=None, trace=False, **opt):
    import torch
    from paper_2602_19699_amd import cbic
    sys_ = cbic.System(ctx, kind, params)
    o = cbic.Options(**opt)
    dev = torch.device("cuda", ctx.device)
    Tt = None if T is None else torch.as_tensor(np.asarray(T, np.int32), device=dev)
    U0t = None if U0 is None else torch.as_tensor(np.asarray(U0, np.float64), device=dev)
    out = cbic.solve_batch(ctx, sys_, torch.as_tensor(np.asarray(x0, np.float64), device=dev), T_max, T=Tt,
                           U0=U0t, opts=o, trace=trace)
    torch.cuda.synchronize(dev)
    res = {k: (None if getattr(out, k) is None else getattr(out, k).cpu().numpy())
           for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx", "xK", "cost_trace", "work")}
    res["status"] = res["status"].astype(np.uint32)
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


def compare(g, r, idx=None, tol_J=1e-9, tol_traj=None, check_status=True, label=""):
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
        # which condition ended the solve must agree; on flat converged instances the
        # last 1-ulp improvements may be accepted by one side and not the other
        same = sg == r.status
        assert same.mean() >= 0.95, f"{label}: status agreement {same.mean():.3f}"
    return float(e[finite].max()) if finite.any() else 0.0


def workload(name, B=None, sys_seed=0):
    return I.workload(name, B=B, sys_seed=sys_seed)


def oracle_with_sensitivity(kind, params, x0, T_max, T=None, opts=None):
    """Oracle solve plus its own sensitivity: the largest relative change of J
    when x0 is perturbed by one ulp either way.  Instances whose result moves
    by more than ~1e-11 under such a perturbation are ill-conditioned under
    rounding (chaotic closed-loop rollouts); no two FP64 implementations can
    agree on them to 1e-9, so they are checked for validity instead."""
    r = orc.solve_batch(kind, params, x0, T_max, T=T, opts=opts)
    rho = np.zeros(len(x0))
    for f in (1 + 2.0 ** -52, 1 - 2.0 ** -53):
        rp = orc.solve_batch(kind, params, x0 * f, T_max, T=T, opts=opts)
        rho = np.maximum(rho, np.where(np.isfinite(r.J), rel(rp.J, r.J), 0.0))
    return r, rho


def compare_sensitivity_aware(g, r, rho, idx=None, tol_J=1e-9, well_tol=1e-11, min_well=0.7, label=""):
    idx = np.arange(len(r.J)) if idx is None else np.asarray(idx)
    e = rel(g["J"][idx], r.J)
    well = rho <= well_tol
    bad = np.where(well & (e > tol_J))[0]
    print(f"{label}: {well.sum()}/{len(well)} well-conditioned, max rel there "
          f"{(e[well].max() if well.any() else 0):.2e}; sensitive ones: median rel {np.median(e[~well]) if (~well).any() else 0:.2e}"
          f" vs their own 1-ulp sensitivity median {np.median(rho[~well]) if (~well).any() else 0:.2e}")
    assert len(bad) == 0, f"{label}: {len(bad)} well-conditioned instances beyond {tol_J:g}: worst {e[bad].max():.3e}"
    assert well.mean() >= min_well, f"{label}: only {well.mean():.2f} well-conditioned"
    assert np.all(np.isfinite(g["J"][idx]) == np.isfinite(r.J))
