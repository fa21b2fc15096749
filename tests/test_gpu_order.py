"""The iteration launches take the instances in an order of expected work
(longest horizon, then highest initial cost first); that order is a
scheduling choice and must change no bit of any output.  Each case is solved
with the default order and with CBIC_FLAG_INPUT_ORDER (the horizon sort's
order) and every output is compared bitwise."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

from gpu_helpers import gpu_solve

pytestmark = pytest.mark.gpu

PM, P3, QUAD = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_QUAD_SYNTH
FIELDS = ("X", "U", "J", "iters", "status", "Vbar", "Vx", "xK", "cost_trace", "work", "jtrace")


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _same(ctx, kind, p, x0, Tmax, T=None, **o):
    from paper_2602_19699_amd import cbic
    a = gpu_solve(ctx, kind, p, x0, Tmax, T=T, trace=True, **o)
    flags = o.pop("flags", 0)
    b = gpu_solve(ctx, kind, p, x0, Tmax, T=T, trace=True, flags=flags | cbic.FLAG_INPUT_ORDER, **o)
    for k in FIELDS:
        if a[k] is not None:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"field {k} with {o}")
    return a


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_order_point_mass(ctx, prec):
    kind, p, x0, T, _ = I.workload("pm16k")
    a = _same(ctx, kind, p, x0[:3000], T, precision=prec, stop_mode=1, rtol=1e-4 if prec else 1e-10)
    assert len(np.unique(a["iters"])) > 2  # instances of different work share the batch


def test_order_point_mass_forms(ctx):
    kind, p, x0, T, _ = I.workload("pm16k")
    x = x0[:700]
    Tb = I.horizons(700, 1, 100, seed=4)
    _same(ctx, kind, p, x, T, T=Tb, precision=1, stop_mode=1, rtol=1e-7, u_max=10.0)
    _same(ctx, kind, p, x, T, regularization=1, max_iter=20)
    _same(ctx, kind, p, x, T, T=Tb, precision=1, max_iter=12, iters_per_launch=3, flags=1)
    _same(ctx, kind, p, x, T, group_lanes=2, max_iter=10)


def test_order_beyond_shared_keys(ctx):
    # more slots than the order kernel keeps keys for in shared memory (16384):
    # the keys are recomputed from the workspace in each pass, for a batch of
    # one horizon (J^0 levels split by the obstacle share) and a ragged one
    kind, p, _, T, _ = I.workload("pm16k")
    B = 16384 + 777
    x = I.point_mass_x0(B, seed=2024)
    _same(ctx, kind, p, x, T, precision=1, stop_mode=1, rtol=1e-4)
    _same(ctx, kind, p, x, T, T=I.horizons(B, 1, 100, seed=5), precision=1, stop_mode=1, rtol=1e-4, max_iter=8)


def test_order_arm_ragged(ctx):
    B = 130
    p = I.planar3_params(0)
    x0 = I.planar3_x0(B, 11)
    Tb = I.horizons(B, 50, 200, seed=12)
    _same(ctx, P3, p, x0, 200, T=Tb, max_iter=20)
    _same(ctx, P3, p, x0, 200, T=Tb, precision=1, stop_mode=1, rtol=1e-7, max_iter=40)


def test_order_quadruped(ctx):
    p = I.quad_params(0)
    x0 = I.quad_x0(12, p, seed=7)
    Tb = np.array([40, 12, 33, 40, 5, 27, 40, 18, 40, 1, 22, 39], np.int32)
    _same(ctx, QUAD, p, x0, 40, T=Tb, precision=1, stop_mode=1, rtol=1e-7, max_iter=10)
    _same(ctx, QUAD, p, x0, 40, T=Tb, max_iter=6, u_max=5.0)


def _same_fused(ctx, kind, p, x0, Tmax, T=None, **o):
    # a solve in one launch finalises each slot inside the iteration kernel
    # (also when timed); one iteration per launch takes the iteration launches
    # and a finalisation kernel of its own
    from paper_2602_19699_amd import cbic
    a = gpu_solve(ctx, kind, p, x0, Tmax, T=T, trace=True, **o)
    t = gpu_solve(ctx, kind, p, x0, Tmax, T=T, trace=True, flags=cbic.FLAG_TIMING, **o)
    b = gpu_solve(ctx, kind, p, x0, Tmax, T=T, trace=True, iters_per_launch=1, **o)
    for k in FIELDS:
        if a[k] is not None:
            np.testing.assert_array_equal(a[k], t[k], err_msg=f"field {k} with {o}, timed")
    for k in FIELDS:
        if a[k] is not None:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"field {k} with {o}")


def test_fused_finalisation_point_mass(ctx):
    kind, p, x0, T, _ = I.workload("pm16k")
    x = x0[:1500]
    Tb = I.horizons(1500, 1, 100, seed=8)
    _same_fused(ctx, kind, p, x, T, precision=1, stop_mode=1, rtol=1e-4)
    _same_fused(ctx, kind, p, x, T, T=Tb, max_iter=30)
    _same_fused(ctx, kind, p, x, T, T=Tb, precision=1, stop_mode=1, rtol=1e-7, u_max=10.0, lookahead_K=17)
    _same_fused(ctx, kind, p, x, T, regularization=1, max_iter=20, group_lanes=4)
    # a budget of zero iterations and invalid horizons are finalised as well
    _same_fused(ctx, kind, p, x[:40], T, max_iter=0)
    Tbad = Tb[:40].copy()
    Tbad[[3, 17]] = [0, 500]
    _same_fused(ctx, kind, p, x[:40], T, T=Tbad, max_iter=5)


def test_fused_finalisation_arm_and_lq(ctx):
    p = I.planar3_params(0)
    x0 = I.planar3_x0(130, 11)
    Tb = I.horizons(130, 50, 200, seed=12)
    _same_fused(ctx, P3, p, x0, 200, T=Tb, max_iter=20)
    _same_fused(ctx, P3, p, x0, 200, T=Tb, precision=1, stop_mode=1, rtol=1e-7, max_iter=40, group_lanes=2)
    q = I.lq_random(4, 2, seed=9, ref=True)
    _same_fused(ctx, I.SYS_LQ, q, I.lq_x0(70, 4), 40, max_iter=3, lookahead_K=10)
