"""The allocation-free solve (cbic_solve_batch_noalloc) against the ordinary
one (cbic_solve_batch) through the C ABI: the same kernels on a fixed device
scratch array instead of the context's workspace, so every output must be the
same bits.  Two calls in a row, the second smaller, so that leftovers of the
first in the shared array would show; sizes beyond the array and the flags it
does not take are refused before any launch."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("X", "U", "J", "iters", "status", "Vbar", "Vx", "xK", "cost_trace", "work", "jtrace")


def _run(ctx, kind, p, x0, T_max, T=None, noalloc=False, **opt):
    import torch
    from paper_2602_19699_amd import cbic
    dev = torch.device("cuda", ctx.device)
    sys_ = cbic.System(ctx, kind, p)
    o = cbic.Options(**opt)
    out = cbic.Outputs.allocate(len(x0), T_max, sys_.n, sys_.m, dev, targets=True, trace_iters=o.max_iter)
    x0t = torch.as_tensor(np.asarray(x0, np.float64), device=dev)
    Tt = None if T is None else torch.as_tensor(np.asarray(T, np.int32), device=dev)
    if noalloc:
        cbic.solve_batch_noalloc(ctx, sys_, x0t, T_max, out, T=Tt, opts=o)
    else:
        cbic.solve_batch(ctx, sys_, x0t, T_max, T=Tt, opts=o, out=out)
    torch.cuda.synchronize(dev)
    res = {f: getattr(out, f).cpu().numpy() for f in FIELDS}
    sys_.close()
    return res


def test_noalloc_matches_the_ordinary_solve_twice():
    from paper_2602_19699_amd import cbic
    ctx = cbic.Context(0)
    cases = [
        # a ragged arm batch in the mixed form (horizon sort in the scratch)
        (I.SYS_PLANAR3, I.planar3_params(0), I.planar3_x0(96, 21), 120, I.horizons(96, 30, 120, seed=8),
         dict(max_iter=12, precision=1)),
        # then a smaller point-mass batch in FP64 with the tolerance stop
        (I.SYS_POINT_MASS, I.point_mass_params(0), I.point_mass_x0(40, 22), 80, None,
         dict(max_iter=30, stop_mode=1, rtol=1e-10)),
    ]
    for kind, p, x0, T_max, T, opt in cases:
        print(f"noalloc case: system {kind}, B={len(x0)}, T_max={T_max}, {opt}", flush=True)
        a = _run(ctx, kind, p, x0, T_max, T, **opt)
        b = _run(ctx, kind, p, x0, T_max, T, noalloc=True, **opt)
        for f in FIELDS:
            np.testing.assert_array_equal(a[f], b[f], err_msg=f)
        assert np.all(np.isfinite(b["J"]))
    ctx.close()


def test_noalloc_refuses_what_it_cannot_hold():
    import torch
    from paper_2602_19699_amd import cbic
    ctx = cbic.Context(0)
    kind, p, x0, T_max, _ = I.workload("pm16k")
    sys_ = cbic.System(ctx, kind, p)
    need = sys_.workspace_size(len(x0), T_max)
    assert need > cbic.NOALLOC_SCRATCH_BYTES
    dev = torch.device("cuda", 0)
    out = cbic.Outputs.allocate(len(x0), T_max, 4, 2, dev)
    x0t = torch.as_tensor(x0, device=dev)
    with pytest.raises(cbic.CbicError) as e:
        cbic.solve_batch_noalloc(ctx, sys_, x0t, T_max, out)
    assert e.value.code == cbic.E_OOM
    small = cbic.Outputs.allocate(8, T_max, 4, 2, dev)
    for flags in (cbic.FLAG_GRAPH, cbic.FLAG_TIMING):
        with pytest.raises(cbic.CbicError) as e:
            cbic.solve_batch_noalloc(ctx, sys_, x0t[:8], T_max, small, opts=cbic.Options(flags=flags))
        assert e.value.code == cbic.E_INVALID
    sys_.close()
    ctx.close()
