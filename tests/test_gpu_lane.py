"""GPU parity of the lane-per-instance solver (point mass, arm, LQ) against the
FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import check_parity, compare, gpu_solve, oracle_ensemble, oracle_opts, rel, trace_sensitivity

pytestmark = pytest.mark.gpu

PM, P3, LQ = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_LQ


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _targets(g, r, idx, label, kind, p, x0, T_max, T=None, K=0, well=None):
    """Critic targets.  (a) Exact: on the GPU's own final trajectory the
    oracle's extraction (no re-simulation) must reproduce V-bar, V-bar_x and
    x_{k+K} to rounding, every step must satisfy the dynamics to rounding and
    the returned J must be that trajectory's cost.  (b) Against the oracle's
    own solution the trajectories agree only to the flatness of the optimum:
    cost differences of ~1e-15 J allow state differences of ~sqrt(1e-15 J / lambda)."""
    idx = np.asarray(idx)
    for j, b in enumerate(idx):
        Tb = T_max if T is None else int(np.asarray(T)[b])
        X, U = g["X"][b, :Tb + 1], g["U"][b, :Tb]
        Vb, Vx, xK = orc.extract(kind, p, X, U, K)
        sc = np.abs(Vb).max()
        assert np.abs(g["Vbar"][b, :Tb + 1] - Vb).max() <= 1e-12 * sc, f"{label}: Vbar (exact) #{b}"
        assert np.abs(g["Vx"][b, :Tb + 1] - Vx).max() <= 1e-10 * (np.abs(Vx).max() + 1e-300), f"{label}: Vx #{b}"
        assert np.array_equal(g["xK"][b, :Tb + 1], xK), f"{label}: xK #{b}"
        d, J = orc.check_trajectory(kind, p, X, U)
        assert d <= 1e-12, f"{label}: dynamics residual {d:.2e} #{b}"
        assert abs(g["J"][b] - J) <= 1e-12 * abs(J), f"{label}: J of returned trajectory #{b}"
        assert np.array_equal(X[0], x0[b])
    # (b) against the oracle's solution (r holds the whole batch), where the
    # instance is not sensitive to rounding
    if well is not None:
        idx = idx[np.asarray(well)[idx]]
    scale = np.abs(r.Vbar[idx]).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(g["Vbar"][idx] - r.Vbar[idx]) <= 1e-6 * scale), f"{label}: Vbar"
    sx = np.abs(r.Vx[idx]).max(axis=(1, 2), keepdims=True) + 1.0
    assert np.all(np.abs(g["Vx"][idx] - r.Vx[idx]) <= 1e-5 * sx), f"{label}: Vx"
    assert np.all(np.abs(g["xK"][idx] - r.xK[idx]) <= 1e-5 * (1 + np.abs(r.xK[idx]))), f"{label}: xK"


def test_point_mass_64_fp64(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    g = gpu_solve(ctx, kind, p, x0, T, trace=True)
    r = orc.solve_batch(kind, p, x0, T, opts=oracle_opts())
    worst = compare(g, r, label="pm64")
    print(f"pm64 fp64 worst rel cost {worst:.2e}; iters gpu {g['iters'][:8]} oracle {r.iters[:8]}")
    np.testing.assert_allclose(g["X"], r.X, atol=1e-5)
    _targets(g, r, np.arange(64), "pm64", kind, p, x0, T)
    # accepted steps strictly lower the cost (GPU trace)
    for b in range(64):
        tr = g["cost_trace"][b, : g["iters"][b] + 1]
        assert np.all(np.diff(tr) < 0)


def test_point_mass_ragged_multi_wave_fp64(ctx):
    # 200 instances = three full waves and a ragged tail; horizons 1..100
    B = 200
    p = I.point_mass_params(1)
    x0 = I.point_mass_x0(B, 77)
    T = I.horizons(B, 1, 100, seed=5)
    g = gpu_solve(ctx, PM, p, x0, 100, T=T, lookahead_K=7)
    r = orc.solve_batch(PM, p, x0, 100, T=T, opts=oracle_opts(lookahead_K=7))
    compare(g, r, label="pm-ragged")
    _targets(g, r, np.arange(B), "pm-ragged", PM, p, x0, 100, T=T, K=7)
    for b in range(B):
        assert np.all(g["X"][b, T[b] + 1:] == 0) and np.all(g["U"][b, T[b]:] == 0)


def test_point_mass_16k_sampled_fp64(ctx):
    kind, p, x0, T, _ = I.workload("pm16k")
    g = gpu_solve(ctx, kind, p, x0, T)
    idx = np.random.default_rng(0).choice(len(x0), 96, replace=False)
    idx = np.r_[idx, [0, len(x0) - 1]]
    r = orc.solve_batch(kind, p, x0[idx], T, opts=oracle_opts())
    compare(g, r, idx=idx, label="pm16k")
    assert np.all(np.isfinite(g["J"]))
    assert np.all((g["status"] & (orc.ST_NONFINITE | orc.ST_CHOL_FAIL)) == 0)


def test_point_mass_16k_headline_form(ctx):
    # the timed configuration: all 16384 instances, mixed form, relative-decrease
    # stop at 1e-4, default launch options; every instance ended by its stop
    # rule within 1e-4 of the FP64 oracle's cost, and a second solve bitwise
    # identical
    kind, p, x0, T, _ = I.workload("pm16k")
    opts = dict(precision=1, stop_mode=1, rtol=1e-4)
    g = gpu_solve(ctx, kind, p, x0, T, **opts)
    r = orc.solve_batch(kind, p, x0, T, opts=oracle_opts())
    e = rel(g["J"], r.J)
    print(f"pm16k headline form: max rel {e.max():.2e}, median {np.median(e):.2e}")
    assert e.max() <= 1e-4
    assert np.all((g["status"] & (orc.ST_NONFINITE | orc.ST_CHOL_FAIL | orc.ST_MAX_ITER)) == 0)
    g2 = gpu_solve(ctx, kind, p, x0, T, **opts)
    for f in ("J", "X", "U", "iters", "status", "Vbar", "Vx"):
        np.testing.assert_array_equal(g[f], g2[f], err_msg=f)


def test_point_mass_mixed_precision(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    g = gpu_solve(ctx, kind, p, x0, T, precision=1)
    r = orc.solve_batch(kind, p, x0, T, opts=oracle_opts())
    e = rel(g["J"], r.J)
    print(f"pm64 mixed: max rel {e.max():.2e}")
    assert np.all(e <= 1e-4)
    assert np.all(np.isfinite(g["J"]))


def test_point_mass_tolerance_mode(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    g = gpu_solve(ctx, kind, p, x0, T, stop_mode=1, rtol=1e-10)
    r = orc.solve_batch(kind, p, x0, T, opts=oracle_opts(stop_mode=1, rtol=1e-10))
    compare(g, r, label="pm-tol")
    assert np.mean((g["status"] & orc.ST_CONVERGED) > 0) > 0.5


@pytest.mark.parametrize("n,m", [(2, 1), (4, 2), (6, 3)])
def test_lq_one_iteration_optimum(ctx, n, m):
    p = I.lq_random(n, m, seed=n, ref=True)
    x0 = I.lq_x0(70, n)
    T = 40
    U0 = np.random.default_rng(1).normal(size=(70, T, m))
    g = gpu_solve(ctx, LQ, p, x0, T, U0=U0, max_iter=1)
    r = orc.solve_batch(LQ, p, x0, T, U0=U0, opts=oracle_opts(max_iter=1))
    compare(g, r, tol_J=1e-11, label=f"lq{n}{m}")
    np.testing.assert_allclose(g["U"], r.U, atol=1e-9)


def test_lq_clip_floors_alternate(ctx):
    # an LQ system's clipped constant Hessians depend on psd_eps: solves with
    # different floors, in any order, each match the oracle under their own
    # floor, and repeating a floor repeats its bits
    q = I.lq_random(4, 2, seed=5, ref=True)
    x0 = I.lq_x0(20, 4, seed=3)
    runs = {}
    for eps in (1e-6, 0.7, 1e-6, 0.7, 0.0):
        g = gpu_solve(ctx, LQ, q, x0, 30, max_iter=3, psd_eps=eps)
        r = orc.solve_batch(LQ, q, x0, 30, opts=oracle_opts(max_iter=3, psd_eps=eps))
        compare(g, r, tol_J=1e-11, label=f"lq eps={eps}")
        if eps in runs:
            np.testing.assert_array_equal(runs[eps]["U"], g["U"])
        runs[eps] = g
    assert not np.array_equal(runs[1e-6]["U"], runs[0.7]["U"])


def test_arm_ragged_fp64(ctx):
    # per instance: equal to the oracle to 1e-9, or a near-tie line-search
    # decision replayed, or rounding-sensitive (its own cost moves under a
    # one-ulp change of x0) with the prefix before the onset equal and the
    # result valid (check_parity)
    B = 130
    p = I.planar3_params(0)
    x0 = I.planar3_x0(B, 11)
    T = I.horizons(B, 50, 200, seed=12)
    for it in (1, 20):
        g = gpu_solve(ctx, P3, p, x0, 200, T=T, max_iter=it, trace=True)
        o = oracle_opts(max_iter=it)
        r, rps = oracle_ensemble(P3, p, x0, 200, T=T, opts=o)
        check_parity(g, P3, p, x0, 200, T, o, r, rps, label=f"arm {it} it")
        # critic targets: exact on every returned trajectory; against the
        # oracle's solution where the instance is not sensitive to rounding
        well = trace_sensitivity(r, rps)[:, -1] <= 1e-11
        _targets(g, r, np.arange(B), f"arm {it} it", P3, p, x0, 200, T=T, well=well)
        _replay_all(g, P3, p, x0, 200, T)


def _replay_all(g, kind, p, x0, T_max, T):
    # every returned trajectory satisfies the dynamics step by step and has the returned cost
    for b in range(len(x0)):
        Tb = T_max if T is None else int(T[b])
        d, J = orc.check_trajectory(kind, p, g["X"][b, :Tb + 1], g["U"][b, :Tb])
        assert d <= 1e-12 and abs(J - g["J"][b]) <= 1e-12 * abs(J), f"instance {b}: residual {d:.2e}"
        assert np.array_equal(g["X"][b, 0], x0[b])


def test_arm_4k_sampled(ctx):
    # the arm workload at full size (4096 instances, horizons 50..200, FP64,
    # 50 iterations); 512 instances checked against the oracle per instance
    kind, p, x0, T, Tb = I.workload("arm4k")
    g = gpu_solve(ctx, kind, p, x0, T, T=Tb, trace=True)
    idx = np.r_[np.random.default_rng(1).choice(np.arange(1, len(x0) - 1), 510, replace=False), 0, len(x0) - 1]
    o = oracle_opts()
    r, rps = oracle_ensemble(kind, p, x0[idx], T, T=Tb[idx], opts=o)
    sets = check_parity(g, kind, p, x0, T, Tb, o, r, rps, idx=idx, label="arm4k fp64")
    assert sum(sets.values()) == len(idx)
    _replay_all({k: (v[idx] if v is not None else None) for k, v in g.items()}, kind, p, x0[idx], T, Tb[idx])


@pytest.mark.parametrize("umax", [np.inf, 8.0], ids=["unbounded", "umax8"])
def test_arm_4k_mixed(ctx, umax):
    # the arm's mixed form (FP32 rollouts, derivatives and Riccati products;
    # FP64 Cholesky, cost sums and line-search comparison) with the tolerance
    # stop, against the FP64 oracle at 1e-4 on 512 instances of the full
    # workload; the rounding-sensitive set is measured with perturbations of
    # one FP32 rounding (2^-24) of x0
    kind, p, x0, T, Tb = I.workload("arm4k")
    g = gpu_solve(ctx, kind, p, x0, T, T=Tb, trace=True, precision=1, stop_mode=1, rtol=1e-7, u_max=umax)
    idx = np.r_[np.random.default_rng(2).choice(np.arange(1, len(x0) - 1), 510, replace=False), 0, len(x0) - 1]
    o = oracle_opts(stop_mode=1, rtol=1e-7, u_max=umax)
    r, rps = oracle_ensemble(kind, p, x0[idx], T, T=Tb[idx], opts=o, rel_step=2.0 ** -24, probe32=True)
    check_parity(g, kind, p, x0, T, Tb, o, r, rps, idx=idx, tol=1e-4, onset_tol=1e-6, mixed=True,
                 label=f"arm4k mixed u_max={umax}")


def test_edge_cases(ctx):
    p = I.point_mass_params(0)
    x0 = I.point_mass_x0(5, 3)
    x0[2, 1] = np.nan
    # one instance, horizon 1
    g = gpu_solve(ctx, PM, p, x0[:1], 1)
    r = orc.solve_batch(PM, p, x0[:1], 1, opts=oracle_opts())
    compare(g, r, label="T=1")
    # NaN initial state: frozen NONFINITE, others unaffected
    g = gpu_solve(ctx, PM, p, x0, 30)
    r = orc.solve_batch(PM, p, x0, 30, opts=oracle_opts())
    assert g["status"][2] == orc.ST_NONFINITE and g["iters"][2] == 0
    ok = [0, 1, 3, 4]
    assert np.all(rel(g["J"][ok], r.J[ok]) <= 1e-9)
    # no line-search trials: LS_FAILED immediately, zero controls returned
    g = gpu_solve(ctx, PM, p, x0[:2], 30, ls_max_trials=0)
    assert np.all(g["status"] == orc.ST_LS_FAILED) and np.all(g["U"] == 0)
    # zero budget
    g = gpu_solve(ctx, PM, p, x0[:2], 30, max_iter=0)
    assert np.all(g["status"] == orc.ST_MAX_ITER) and np.all(g["iters"] == 0)
    # horizons outside 1..T_max are flagged on the device and never indexed
    g = gpu_solve(ctx, PM, p, x0[[0, 1, 3]], 30, T=np.array([5, 0, 31], np.int32))
    assert g["status"][0] & orc.ST_LS_FAILED or g["status"][0] & orc.ST_MAX_ITER
    assert g["status"][1] == 32 and g["status"][2] == 32
    assert np.isnan(g["J"][1]) and np.all(g["X"][1:] == 0) and np.all(g["U"][1:] == 0)
    # Cholesky failure: indefinite control cost clipped to 0 and no control authority
    lq = I.lq_params(np.eye(2), np.zeros((2, 1)), np.eye(2), -np.eye(1), np.eye(2))
    g = gpu_solve(ctx, LQ, lq, np.ones((1, 2)), 5, psd_eps=0.0)
    assert g["status"][0] == orc.ST_CHOL_FAIL and g["iters"][0] == 0


def test_chunked_and_graph_launches_match_single_launch(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    a = gpu_solve(ctx, kind, p, x0, T)
    b = gpu_solve(ctx, kind, p, x0, T, iters_per_launch=3)
    c = gpu_solve(ctx, kind, p, x0, T, iters_per_launch=5, flags=1)
    c2 = gpu_solve(ctx, kind, p, x0, T, iters_per_launch=5, flags=1)  # graph replay from the cache
    for other in (b, c, c2):
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(a[k], other[k])


def test_batch_independence(ctx):
    p = I.planar3_params(0)
    x0 = I.planar3_x0(70, 4)
    T = I.horizons(70, 10, 60, seed=9)
    full = gpu_solve(ctx, P3, p, x0, 60, T=T, max_iter=10)
    for b in (0, 33, 69):
        one = gpu_solve(ctx, P3, p, x0[[b]], int(T[b]), max_iter=10)
        assert one["J"][0] == full["J"][b]
        np.testing.assert_array_equal(one["X"][0], full["X"][b, : T[b] + 1])


@pytest.mark.parametrize("kind", [PM, P3], ids=["pm", "arm"])
def test_group_widths_give_identical_results(ctx, kind):
    # lanes of a group split the line-search trials; the first accepted step is
    # the same as in the sequential rule, so results are bitwise identical
    if kind == PM:
        p, x0, T, Tb = I.point_mass_params(0), I.point_mass_x0(150, 5), 100, None
    else:
        p, x0, T, Tb = I.planar3_params(0), I.planar3_x0(90, 6), 120, I.horizons(90, 30, 120, seed=3)
    ref = gpu_solve(ctx, kind, p, x0, T, T=Tb, max_iter=15, group_lanes=1)
    for gl in (2, 4, 8, 16):
        g = gpu_solve(ctx, kind, p, x0, T, T=Tb, max_iter=15, group_lanes=gl)
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(ref[k], g[k], err_msg=f"group_lanes={gl} field {k}")


@pytest.mark.parametrize("kind", [PM, P3], ids=["pm", "arm"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("K", [0, 7], ids=["full", "K7"])
def test_partial_targets_identical(ctx, kind, prec, K):
    # every subset of the critic targets (V-bar, V-bar_x, x_{k+K}) is the same
    # bits as the full request: the finalize kernel takes other branches when
    # some are not requested (the costate walk, the stage costs and the sums)
    import torch
    from paper_2602_19699_amd import cbic
    if kind == PM:
        p, x0, T_max, Tb = I.point_mass_params(0), I.point_mass_x0(100, 31), 60, I.horizons(100, 1, 60, seed=2)
    else:
        p, x0, T_max, Tb = I.planar3_params(0), I.planar3_x0(40, 32), 80, I.horizons(40, 20, 80, seed=4)
    dev = torch.device("cuda", ctx.device)
    sys_ = cbic.System(ctx, kind, p)
    o = cbic.Options(max_iter=10, precision=prec, lookahead_K=K)
    x0t = torch.as_tensor(x0, device=dev)
    Tt = torch.as_tensor(Tb, device=dev)
    B = len(x0)

    def run(**keep):
        out = cbic.Outputs.allocate(B, T_max, sys_.n, sys_.m, dev, targets=True)
        for f in ("Vbar", "Vx", "xK"):
            if not keep.get(f, False):
                setattr(out, f, None)
        cbic.solve_batch(ctx, sys_, x0t, T_max, T=Tt, opts=o, out=out)
        torch.cuda.synchronize(dev)
        return {f: None if getattr(out, f) is None else getattr(out, f).cpu().numpy()
                for f in ("X", "U", "J", "Vbar", "Vx", "xK")}

    full = run(Vbar=True, Vx=True, xK=True)
    for keep in (dict(Vbar=True), dict(Vx=True), dict(xK=True), dict(Vbar=True, xK=True), {}):
        part = run(**keep)
        for f, v in part.items():
            if v is not None:
                np.testing.assert_array_equal(v, full[f], err_msg=f"{keep} field {f}")
    sys_.close()


@pytest.mark.parametrize("kind", [PM, P3], ids=["pm", "arm"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_cholesky_failure_inside_a_chunk(ctx, kind, prec):
    # zero cost weights and a zero clipping floor make Q_uu = 0 at the sweep's
    # first step: the kernel records the failure, finishes the chunk and freezes
    # the instance with its warm start and status CHOL_FAIL, as the oracle does
    # (the point mass takes the axis-pair step, the arm the factored one)
    B, T = 20, 40
    if kind == PM:
        p = I.point_mass_params(0, w_u=0.0)
        p[2:5] = 0.0  # position, terminal and obstacle weights
        x0, m = I.point_mass_x0(B, 5), 2
    else:
        p = I.planar3_params(0, w_u=0.0, w_ee=0.0, w_T=0.0, w_obs=0.0)
        x0, m = I.planar3_x0(B, 6), 3
    U0 = np.random.default_rng(1).normal(size=(B, T, m)) * 0.1
    r = orc.solve_batch(kind, p, x0, T, U0=U0, opts=oracle_opts(psd_eps=0.0))
    assert np.all(r.status == orc.ST_CHOL_FAIL) and np.all(r.iters == 0)
    Uw = U0 if prec == 0 else U0.astype(np.float32).astype(np.float64)
    for gl in (1, 2, 8):
        g = gpu_solve(ctx, kind, p, x0, T, U0=U0, psd_eps=0.0, precision=prec, group_lanes=gl)
        assert np.all(g["status"] == orc.ST_CHOL_FAIL), (gl, g["status"])
        assert np.all(g["iters"] == 0)
        np.testing.assert_array_equal(g["U"], Uw)
