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
