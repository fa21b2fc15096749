"""GPU parity of the control bound |u_k,i| <= u_max (eq. 1) against the FP64
CPU oracle, through the C ABI: bounded control steps in the backward sweep,
clamped rollouts and warm starts."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import check_parity, compare, gpu_solve, oracle_ensemble, oracle_opts, rel
from lq_dense import bounded_qp, dense_qp

pytestmark = pytest.mark.gpu

PM, P3, LQ, QUAD = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_LQ, I.SYS_QUAD_SYNTH


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _feasible(g, umax, T=None):
    U = g["U"]
    assert np.all(np.abs(U) <= umax), f"max |u| {np.abs(U).max()}"


def test_bounded_point_mass_fp64(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    for o in (dict(max_iter=50, u_max=10.0), dict(max_iter=200, stop_mode=1, rtol=1e-10, u_max=10.0)):
        g = gpu_solve(ctx, kind, p, x0, T, trace=True, **o)
        oo = oracle_opts(**o)
        r, rps = oracle_ensemble(kind, p, x0, T, opts=oo)
        check_parity(g, kind, p, x0, T, None, oo, r, rps, label=f"pm64 bounded {o}")
        _feasible(g, 10.0)
        assert np.mean(np.any(np.abs(g["U"]) == 10.0, axis=(1, 2))) > 0.5  # the bound binds
        for b in range(64):
            tr = g["cost_trace"][b, : g["iters"][b] + 1]
            assert np.all(np.diff(tr) < 0)


def test_bounded_point_mass_ragged_and_mixed(ctx):
    B = 200
    p = I.point_mass_params(1)
    x0 = I.point_mass_x0(B, 77)
    T = I.horizons(B, 1, 100, seed=5)
    g = gpu_solve(ctx, PM, p, x0, 100, T=T, u_max=8.0, trace=True)
    o = oracle_opts(u_max=8.0)
    r, rps = oracle_ensemble(PM, p, x0, 100, T=T, opts=o)
    check_parity(g, PM, p, x0, 100, T, o, r, rps, label="pm-ragged bounded")
    _feasible(g, 8.0)
    for b in range(B):
        assert np.all(g["X"][b, T[b] + 1:] == 0) and np.all(g["U"][b, T[b]:] == 0)
    gm = gpu_solve(ctx, PM, p, x0, 100, T=T, precision=1, u_max=8.0, trace=True)
    r32, rps32 = oracle_ensemble(PM, p, x0, 100, T=T, opts=o, rel_step=2.0 ** -24, probe32=True)
    check_parity(gm, PM, p, x0, 100, T, o, r32, rps32, tol=1e-4, onset_tol=1e-6, mixed=True,
                 label="pm-ragged bounded mixed")
    assert np.all(np.isfinite(gm["J"]))
    _feasible(gm, 8.0)


def test_bounded_lq(ctx):
    p = I.lq_random(4, 2, seed=3, ref=True)
    x0 = I.lq_x0(70, 4, seed=8) * 4.0
    # T = 1: one step is the bounded QP's minimiser
    g = gpu_solve(ctx, LQ, p, x0, 1, max_iter=1, u_max=0.4)
    r = orc.solve_batch(LQ, p, x0, 1, opts=oracle_opts(max_iter=1, u_max=0.4))
    np.testing.assert_allclose(g["U"], r.U, atol=1e-12, rtol=0)
    for b in range(0, 70, 7):
        H, g0, J = dense_qp(p, x0[b], 1)
        np.testing.assert_allclose(g["U"][b, 0], bounded_qp(H, g0, np.full(2, -0.4), np.full(2, 0.4)), atol=1e-12)
    # T = 12: converged to the bounded QP's minimiser
    q = I.lq_random(4, 2, seed=9, ref=True)
    x1 = I.lq_x0(8, 4, seed=5) * 3.0
    g = gpu_solve(ctx, LQ, q, x1, 12, max_iter=100, stop_mode=1, rtol=1e-15, u_max=0.15)
    for b in range(8):
        H, g0, J = dense_qp(q, x1[b], 12)
        u = bounded_qp(H, g0, np.full(24, -0.15), np.full(24, 0.15))
        assert abs(g["J"][b] - J(u)) <= 1e-11 * abs(J(u))
        np.testing.assert_allclose(g["U"][b].ravel(), u, atol=1e-6, rtol=0)


def test_bounded_arm_ragged_fp64(ctx):
    B = 130
    p = I.planar3_params(0)
    x0 = I.planar3_x0(B, 11)
    T = I.horizons(B, 50, 200, seed=12)
    g = gpu_solve(ctx, P3, p, x0, 200, T=T, max_iter=20, u_max=8.0, trace=True)
    o = oracle_opts(max_iter=20, u_max=8.0)
    r, rps = oracle_ensemble(P3, p, x0, 200, T=T, opts=o)
    check_parity(g, P3, p, x0, 200, T, o, r, rps, label="arm bounded")
    _feasible(g, 8.0)
    for b in range(B):
        d, J = orc.check_trajectory(P3, p, g["X"][b, :T[b] + 1], g["U"][b, :T[b]])
        assert d <= 1e-12 and abs(J - g["J"][b]) <= 1e-12 * abs(J)


def test_bounded_16k_sampled_and_feasible(ctx):
    kind, p, x0, T, _ = I.workload("pm16k")
    g = gpu_solve(ctx, kind, p, x0, T, u_max=10.0, trace=True)
    _feasible(g, 10.0)
    idx = np.r_[np.random.default_rng(4).choice(np.arange(1, len(x0) - 1), 254, replace=False), 0, len(x0) - 1]
    o = oracle_opts(u_max=10.0)
    r, rps = oracle_ensemble(kind, p, x0[idx], T, opts=o)
    check_parity(g, kind, p, x0, T, None, o, r, rps, idx=idx, label="pm16k bounded")


@pytest.mark.parametrize("kind", [PM, P3], ids=["pm", "arm"])
def test_bounded_group_widths_and_launch_splits_identical(ctx, kind):
    if kind == PM:
        p, x0, T, Tb, um = I.point_mass_params(0), I.point_mass_x0(150, 5), 100, None, 10.0
    else:
        p, x0, T, Tb, um = I.planar3_params(0), I.planar3_x0(90, 6), 120, I.horizons(90, 30, 120, seed=3), 8.0
    ref = gpu_solve(ctx, kind, p, x0, T, T=Tb, max_iter=15, group_lanes=1, u_max=um)
    runs = [dict(group_lanes=gl) for gl in (2, 4, 8, 16)]
    runs += [dict(group_lanes=1, iters_per_launch=4), dict(group_lanes=1, iters_per_launch=5, flags=1)]
    for o in runs:
        g = gpu_solve(ctx, kind, p, x0, T, T=Tb, max_iter=15, u_max=um, **o)
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(ref[k], g[k], err_msg=f"{o} field {k}")


def test_loose_bound_and_warm_start(ctx):
    # the bounded kernel with a bound that never binds gives the unbounded kernel's bits
    kind, p, x0, T, _ = I.workload("pm64")
    for prec in (0, 1):
        a = gpu_solve(ctx, kind, p, x0, T, max_iter=20, precision=prec)
        b = gpu_solve(ctx, kind, p, x0, T, max_iter=20, precision=prec, u_max=1e30)
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"precision {prec} field {k}")
    # the warm start is clamped into the box
    U0 = np.random.default_rng(2).normal(size=(64, T, 2)) * 10.0
    g = gpu_solve(ctx, kind, p, x0, T, U0=U0, max_iter=0, u_max=5.0)
    r = orc.solve_batch(kind, p, x0, T, U0=U0, opts=oracle_opts(max_iter=0, u_max=5.0))
    np.testing.assert_array_equal(g["U"], np.clip(U0, -5.0, 5.0))
    assert np.all(rel(g["J"], r.J) <= 1e-13)


def test_bounded_with_levenberg_marquardt(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    o = dict(max_iter=50, u_max=10.0, regularization=1)
    g = gpu_solve(ctx, kind, p, x0, T, trace=True, **o)
    oo = oracle_opts(**o)
    r, rps = oracle_ensemble(kind, p, x0, T, opts=oo)
    check_parity(g, kind, p, x0, T, None, oo, r, rps, label="pm64 bounded LM")
    _feasible(g, 10.0)


def test_invalid_bounds_rejected(ctx):
    from paper_2602_19699_amd import cbic
    kind, p, x0, T, _ = I.workload("pm64")
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(cbic.CbicError) as e:
            gpu_solve(ctx, kind, p, x0[:2], T, u_max=bad)
        assert e.value.code == cbic.E_INVALID


def _quad_case():
    p = I.quad_params(0)
    return p, I.quad_x0(8, p, seed=7), np.array([40, 12, 33, 40, 5, 27, 40, 18], np.int32)


def test_bounded_quadruped(ctx):
    # the workgroup kernel's bounded step (the FP64 box QP on wave 0, the
    # feedback rows of the free components from the face factor) and clamped
    # rollouts, against the oracle in both forms
    p, x0, T = _quad_case()
    for um in (5.0, 2.0):
        o = dict(max_iter=12, u_max=um)
        g = gpu_solve(ctx, QUAD, p, x0, 40, T=T, trace=True, **o)
        oo = oracle_opts(**o)
        r, rps = oracle_ensemble(QUAD, p, x0, 40, T=T, opts=oo)
        check_parity(g, QUAD, p, x0, 40, T, oo, r, rps, label=f"quad bounded {um}")
        _feasible(g, um)
        assert np.mean(np.abs(g["U"]) == um) > 0.05  # the bound binds
    o = dict(max_iter=12, u_max=5.0)
    gm = gpu_solve(ctx, QUAD, p, x0, 40, T=T, trace=True, precision=1, **o)
    oo = oracle_opts(**o)
    r32, rps32 = oracle_ensemble(QUAD, p, x0, 40, T=T, opts=oo, rel_step=2.0 ** -24, probe32=True)
    check_parity(gm, QUAD, p, x0, 40, T, oo, r32, rps32, tol=1e-4, onset_tol=1e-6, mixed=True,
                 label="quad bounded mixed")
    _feasible(gm, 5.0)


def test_bounded_quadruped_loose_bound_warm_start_and_launch_splits(ctx):
    p, x0, T = _quad_case()
    for prec in (0, 1):
        a = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=8, precision=prec)
        b = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=8, precision=prec, u_max=1e30)
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"precision {prec} field {k}")
        c = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=8, precision=prec, u_max=4.0)
        d = gpu_solve(ctx, QUAD, p, x0, 40, T=T, max_iter=8, precision=prec, u_max=4.0, iters_per_launch=3)
        for k in ("X", "U", "J", "iters", "status", "Vbar", "Vx"):
            np.testing.assert_array_equal(c[k], d[k], err_msg=f"launch split, precision {prec} field {k}")
    U0 = np.random.default_rng(2).normal(size=(8, 40, 12)) * 10.0
    g = gpu_solve(ctx, QUAD, p, x0, 40, T=T, U0=U0, max_iter=0, u_max=5.0)
    r = orc.solve_batch(QUAD, p, x0, 40, T=T, U0=U0, opts=oracle_opts(max_iter=0, u_max=5.0))
    for b in range(8):
        np.testing.assert_array_equal(g["U"][b, :T[b]], np.clip(U0[b, :T[b]], -5.0, 5.0))
    assert np.all(rel(g["J"], r.J) <= 1e-13)
