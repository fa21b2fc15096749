"""GPU parity of the workgroup-per-instance solver for the 37-state synthetic
quadruped against the FP64 CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import compare, gpu_solve, oracle_opts, rel

pytestmark = pytest.mark.gpu

QUAD = I.SYS_QUAD_SYNTH


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _check_targets(g, kind, p, x0, T, idx):
    for b in idx:
        X, U = g["X"][b, :T + 1], g["U"][b, :T]
        Vb, Vx, xK = orc.extract(kind, p, X, U)
        assert np.abs(g["Vbar"][b] - Vb).max() <= 1e-11 * np.abs(Vb).max()
        assert np.abs(g["Vx"][b] - Vx).max() <= 1e-9 * (np.abs(Vx).max() + 1e-300)
        assert np.array_equal(g["xK"][b], xK)
        d, J = orc.check_trajectory(kind, p, X, U)
        assert d <= 1e-12 and abs(J - g["J"][b]) <= 1e-12 * abs(J)


def test_quad_small_fp64_and_ragged(ctx):
    p = I.quad_params(0)
    x0 = I.quad_x0(6, p, seed=7)
    T = np.array([30, 1, 17, 30, 2, 25], np.int32)
    g = gpu_solve(ctx, QUAD, p, x0, 30, T=T, max_iter=12, trace=True)
    r = orc.solve_batch(QUAD, p, x0, 30, T=T, opts=oracle_opts(max_iter=12))
    worst = compare(g, r, label="quad-small")
    print(f"quad fp64 worst rel cost {worst:.2e}; iters {g['iters']} vs {r.iters}; status {g['status']}")
    for b in range(6):
        tr = g["cost_trace"][b, : g["iters"][b] + 1]
        assert np.all(np.diff(tr) < 0)
        Tb = int(T[b])
        Vb, Vx, xK = orc.extract(QUAD, p, g["X"][b, :Tb + 1], g["U"][b, :Tb])
        assert np.abs(g["Vbar"][b, :Tb + 1] - Vb).max() <= 1e-11 * np.abs(Vb).max()
        assert np.abs(g["Vx"][b, :Tb + 1] - Vx).max() <= 1e-9 * (np.abs(Vx).max() + 1e-300)
        assert np.all(g["X"][b, Tb + 1:] == 0)


def test_quad_mixed_precision(ctx):
    p = I.quad_params(0)
    x0 = I.quad_x0(8, p, seed=8)
    g = gpu_solve(ctx, QUAD, p, x0, 40, precision=1, stop_mode=1, rtol=1e-7)
    r = orc.solve_batch(QUAD, p, x0, 40, opts=oracle_opts())
    e = rel(g["J"], r.J)
    print(f"quad mixed max rel {e.max():.2e}")
    assert e.max() <= 1e-4


def test_quad_1k_sampled(ctx):
    kind, p, x0, T, _ = I.workload("quad1k")
    g = gpu_solve(ctx, kind, p, x0, T)
    idx = np.r_[np.random.default_rng(2).choice(np.arange(1, len(x0) - 1), 126, replace=False), 0, len(x0) - 1]
    r = orc.solve_batch(kind, p, x0[idx], T, opts=oracle_opts())
    worst = compare(g, r, idx=idx, label="quad1k")
    print(f"quad1k fp64: {len(idx)} instances, max rel cost {worst:.2e}")
    _check_targets(g, kind, p, x0, T, idx[:16])
    assert np.all(np.isfinite(g["J"]))


def test_quad_1k_headline_form(ctx):
    # the timed configuration of the quadruped: 1024 instances, mixed form,
    # relative-decrease stop at 1e-4; every instance against the FP64 oracle
    # at the 1e-4 cost bar, every instance ended by its stop rule
    kind, p, x0, T, _ = I.workload("quad1k")
    g = gpu_solve(ctx, kind, p, x0, T, precision=1, stop_mode=1, rtol=1e-4)
    r = orc.solve_batch(kind, p, x0, T, opts=oracle_opts())
    e = rel(g["J"], r.J)
    print(f"quad1k headline form: {len(e)} instances, max rel {e.max():.2e}, median {np.median(e):.2e}")
    assert e.max() <= 1e-4
    assert np.all((g["status"] & (orc.ST_NONFINITE | orc.ST_CHOL_FAIL | orc.ST_MAX_ITER)) == 0)


def test_quad_edge_cases(ctx):
    p = I.quad_params(0)
    x0 = I.quad_x0(5, p, seed=3)
    x0[2, 1] = np.nan
    # one instance, horizon 1, both forms
    r = orc.solve_batch(QUAD, p, x0[:1], 1, opts=oracle_opts())
    compare(gpu_solve(ctx, QUAD, p, x0[:1], 1), r, label="quad T=1")
    gm = gpu_solve(ctx, QUAD, p, x0[:1], 1, precision=1)
    assert rel(gm["J"], r.J).max() <= 1e-4
    # NaN initial state: frozen NONFINITE, the others unaffected
    g = gpu_solve(ctx, QUAD, p, x0, 20)
    r = orc.solve_batch(QUAD, p, x0, 20, opts=oracle_opts())
    assert g["status"][2] == orc.ST_NONFINITE and g["iters"][2] == 0
    ok = [0, 1, 3, 4]
    assert np.all(rel(g["J"][ok], r.J[ok]) <= 1e-9)
    # no line-search trials: LS_FAILED at once, the zero warm start returned
    g = gpu_solve(ctx, QUAD, p, x0[:2], 20, ls_max_trials=0)
    assert np.all(g["status"] == orc.ST_LS_FAILED) and np.all(g["U"] == 0)
    # zero budget
    g = gpu_solve(ctx, QUAD, p, x0[:2], 20, max_iter=0)
    assert np.all(g["status"] == orc.ST_MAX_ITER) and np.all(g["iters"] == 0)
    # horizons outside 1..T_max are flagged and never indexed
    g = gpu_solve(ctx, QUAD, p, x0[[0, 1, 3]], 20, T=np.array([5, 0, 21], np.int32))
    assert g["status"][1] == 32 and g["status"][2] == 32
    assert np.isnan(g["J"][1]) and np.isnan(g["J"][2])
    assert np.all(g["X"][1:] == 0) and np.all(g["U"][1:] == 0)
    r = orc.solve_batch(QUAD, p, x0[:1], 20, T=np.array([5], np.int32), opts=oracle_opts())
    compare(g, r, idx=[0], label="quad T=5 beside bad horizons")


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_quad_cholesky_failure_keeps_warm_start(ctx, prec):
    # zero cost weights and a zero clipping floor make Q_uu = 0 at the sweep's
    # first step: the instance is frozen with its warm start and CHOL_FAIL, as
    # in the oracle
    B, T = 3, 20
    p = I.quad_params(0, w_u=0.0, w_T=0.0, w_q=0.0, w_v=0.0)
    x0 = I.quad_x0(B, p, seed=4)
    U0 = np.random.default_rng(2).normal(size=(B, T, 12)) * 0.1
    r = orc.solve_batch(QUAD, p, x0, T, U0=U0, opts=oracle_opts(psd_eps=0.0))
    assert np.all(r.status == orc.ST_CHOL_FAIL) and np.all(r.iters == 0)
    g = gpu_solve(ctx, QUAD, p, x0, T, U0=U0, psd_eps=0.0, precision=prec)
    assert np.all(g["status"] == orc.ST_CHOL_FAIL) and np.all(g["iters"] == 0)
    Uw = U0 if prec == 0 else U0.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(g["U"], Uw)


def test_quad_chunk_boundaries(ctx):
    # the sweep evaluates derivative blocks 16 steps at a time and the finalize
    # four: horizons on either side of those boundaries, in one ragged batch
    p = I.quad_params(1)
    T = np.array([15, 16, 17, 32, 33, 3, 4, 5], np.int32)
    x0 = I.quad_x0(len(T), p, seed=9)
    g = gpu_solve(ctx, QUAD, p, x0, 33, T=T)
    r = orc.solve_batch(QUAD, p, x0, 33, T=T, opts=oracle_opts())
    compare(g, r, label="quad chunk boundaries")
    for b in range(len(T)):
        Tb = int(T[b])
        Vb, Vx, xK = orc.extract(QUAD, p, g["X"][b, :Tb + 1], g["U"][b, :Tb])
        assert np.abs(g["Vbar"][b, :Tb + 1] - Vb).max() <= 1e-11 * np.abs(Vb).max()
        assert np.abs(g["Vx"][b, :Tb + 1] - Vx).max() <= 1e-9 * (np.abs(Vx).max() + 1e-300)
        assert np.all(g["X"][b, Tb + 1:] == 0) and np.all(g["U"][b, Tb:] == 0)
    gm = gpu_solve(ctx, QUAD, p, x0, 33, T=T, precision=1, stop_mode=1, rtol=1e-7)
    assert rel(gm["J"], r.J).max() <= 1e-4


def _same(a, b):
    return all(np.array_equal(a[k], b[k], equal_nan=True) for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"))


def test_quad_instances_per_cu(ctx):
    # one or two workgroups per compute unit are register allocations of the
    # same kernel: every form gives the same bits under either, FP64 runs one
    # per unit whatever is asked, and the autotuner's choice (used by solves
    # that leave it at 0) changes nothing either
    import torch
    from paper_2602_19699_amd import cbic
    p = I.quad_params(0)
    x0 = I.quad_x0(8, p, seed=7)
    T = np.array([40, 12, 33, 40, 5, 27, 40, 18], np.int32)
    forms = {"plain": dict(stop_mode=1, rtol=1e-7), "bounded": dict(u_max=5.0),
             "lm": dict(regularization=1), "bounded_lm": dict(u_max=5.0, regularization=1)}
    for name, o in forms.items():
        a = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=12, precision=1, wg_per_cu=1, **o)
        b = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=12, precision=1, wg_per_cu=2, **o)
        c = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=12, precision=1, wg_per_cu=2, iters_per_launch=5, **o)
        assert _same(a, b) and _same(a, c), name
        assert np.all(np.isfinite(a["J"])), name
    a = gpu_solve(ctx, QUAD, p, x0[:3], 20, max_iter=6, wg_per_cu=1)
    b = gpu_solve(ctx, QUAD, p, x0[:3], 20, max_iter=6, wg_per_cu=2)
    assert _same(a, b)
    dev = torch.device("cuda", ctx.device)
    sysm = cbic.System(ctx, QUAD, p)
    try:
        o = cbic.Options(precision=1, stop_mode=1, rtol=1e-4, max_iter=12)
        choice, ms = cbic.autotune(ctx, sysm, torch.as_tensor(x0, device=dev), 40,
                                   T=torch.as_tensor(T, device=dev), opts=o)
        assert choice in (1, 2) and ms > 0
        choice64, _ = cbic.autotune(ctx, sysm, torch.as_tensor(x0, device=dev), 40,
                                    T=torch.as_tensor(T, device=dev), opts=cbic.Options(max_iter=4))
        assert choice64 == 1
    finally:
        sysm.close()
    t = gpu_solve(ctx, QUAD, p, x0, 40, T=T, precision=1, stop_mode=1, rtol=1e-4, max_iter=12)
    u = gpu_solve(ctx, QUAD, p, x0, 40, T=T, precision=1, stop_mode=1, rtol=1e-4, max_iter=12, wg_per_cu=3 - choice)
    assert _same(t, u)
