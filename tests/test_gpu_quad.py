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
    idx = np.r_[np.random.default_rng(2).choice(len(x0), 6, replace=False), 0, len(x0) - 1]
    r = orc.solve_batch(kind, p, x0[idx], T, opts=oracle_opts())
    compare(g, r, idx=idx, label="quad1k")
    _check_targets(g, kind, p, x0, T, idx[:3])
    assert np.all(np.isfinite(g["J"]))
