"""GPU parity of the iteration-budget calibration (paper Sec. IV-A) through
the C ABI: the percentiles and the histogram of per-instance iteration counts
of a relative-decrease-stop solve, against the FP64 oracle on the same
instances."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import gpu_solve

PM, LQ = I.SYS_POINT_MASS, I.SYS_LQ

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _calibrate(ctx, kind, params, x0, T_max, T=None, cap=1000, **opt):
    import torch
    from paper_2602_19699_amd import cbic
    s = cbic.System(ctx, kind, params)
    Tt = None if T is None else torch.as_tensor(np.asarray(T, np.int32), device="cuda")
    out = cbic.calibrate_max_iter(ctx, s, torch.as_tensor(np.asarray(x0, np.float64), device="cuda"), T_max,
                                  T=Tt, opts=cbic.Options(**opt), cap=cap)
    s.close()
    return out


def test_point_mass_matches_oracle(ctx):
    kind, p, x0, T, _ = I.workload("pm64")
    p99, p50, hist = _calibrate(ctx, kind, p, x0, T)
    o99, o50, counts = orc.calibrate_max_iter(kind, p, x0, T, cap=1000)
    oh = np.bincount(counts, minlength=1001)
    assert hist.sum() == len(x0)
    # a count can differ where a last one-ulp improvement is accepted on one
    # side only; the percentiles agree within one iteration
    assert np.abs(hist - oh).sum() <= 4, (np.nonzero(hist - oh), hist[:20], oh[:20])
    assert abs(p99 - o99) <= 1 and abs(p50 - o50) <= 1, (p99, o99, p50, o50)
    # the histogram is that of the same tolerance-stop solve run directly
    g = gpu_solve(ctx, kind, p, x0, T, max_iter=1000, stop_mode=1)
    assert np.array_equal(np.bincount(g["iters"], minlength=1001), hist)


def test_lq_first_iteration_is_final(ctx):
    p = I.lq_random(4, 2, seed=4)
    x0 = I.lq_x0(32, 4)
    p99, p50, hist = _calibrate(ctx, LQ, p, x0, 12)
    assert hist.sum() == 32 and hist[1] + hist[2] == 32 and 1 <= p50 <= p99 <= 2


def test_cap_bad_horizons_and_errors(ctx):
    from paper_2602_19699_amd import cbic
    kind, p, x0, T, _ = I.workload("pm64")
    # a cap of one iteration bounds every count
    p99, p50, hist = _calibrate(ctx, kind, p, x0[:16], T, cap=1)
    assert p99 <= 1 and hist.sum() == 16 and len(hist) == 2
    # an instance with an invalid horizon is left out of the dataset
    Tb = np.full(16, T, np.int32)
    Tb[3] = 0
    p99, p50, hist = _calibrate(ctx, kind, p, x0[:16], T, T=Tb)
    assert hist.sum() == 15
    with pytest.raises(cbic.CbicError):
        _calibrate(ctx, kind, p, x0[:4], T, cap=0)
