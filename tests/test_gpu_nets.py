"""GPU parity of the biased initial-state selection and the actor warm start
(paper Sec. II, III-C/D) against the FP64 oracle, through the C ABI.

The networks compute in FP32 (as the paper's do): network outputs are held to
2e-5 (1 + |y|) against the FP64 oracle (FP32 rounding through at most five
layers of fan-in <= 64; a float32 evaluation of the same networks stays
within 2.1e-6).  The top-N selection is integer work decided on FP32 scores:
it must equal, index for index, the oracle's selection rule applied to the
kernel's own scores, and be valid against the oracle's FP64 scores."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import check_parity, gpu_solve, oracle_ensemble, oracle_opts, rel

pytestmark = pytest.mark.gpu

PM, P3, LQ, QUAD = I.SYS_POINT_MASS, I.SYS_PLANAR3, I.SYS_LQ, I.SYS_QUAD_SYNTH
TOL = 2e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def _nets(in_dim, width, depth, out_dim, seed, act=0, out_act=0, scale=1.0):
    import torch
    from paper_2602_19699_amd import cbic
    params = I.mlp_params(in_dim, width, depth, out_dim, seed=seed)
    g = cbic.Mlp(in_dim, width, depth, out_dim, torch.as_tensor(params, device="cuda"), act, out_act, scale)
    o = orc.Net(in_dim, width, depth, out_dim, act, out_act, scale, params)
    return g, o


def test_mlp_forward_all_shapes(ctx):
    import torch
    from paper_2602_19699_amd import cbic
    rng = np.random.default_rng(0)
    worst = 0.0
    for width in (32, 64):
        for depth in (1, 2, 3, 4):
            for act in (0, 1, 2):
                for out_act in (0, 1, 2):
                    in_dim, out_dim = int(rng.integers(1, 40)), int(rng.integers(1, 17))
                    g, o = _nets(in_dim, width, depth, out_dim, seed=width + 10 * depth + 100 * act + 1000 * out_act,
                                 act=act, out_act=out_act, scale=2.5)
                    x = (rng.normal(size=(333, in_dim)) * 2).astype(np.float32)
                    yg = cbic.mlp_forward(ctx, g, torch.as_tensor(x, device="cuda")).cpu().numpy()
                    yo = orc.mlp_forward(o, x.astype(np.float64))
                    e = np.abs(yg - yo) / (1 + np.abs(yo))
                    worst = max(worst, float(e.max()))
                    assert e.max() <= TOL, (width, depth, act, out_act, e.max())
    print(f"mlp forward: worst error / (1 + |y|) = {worst:.2e}")


@pytest.mark.parametrize("Bc,N", [(163840, 16384), (1000, 100), (1000, 1), (1000, 1000), (1000, 0), (1, 1), (1025, 517)])
def test_bic_select(ctx, Bc, N):
    import torch
    from paper_2602_19699_amd import cbic
    x, T, T_max = I.bic_candidates("pm16k", Bc, seed=17)
    g, o = _nets(5, 64, 3, 1, seed=5, act=0, out_act=2)
    sg, sel, xs, Ts = cbic.bic_select(ctx, g, torch.as_tensor(x, device="cuda"), torch.as_tensor(T, device="cuda"),
                                      T_max, N, gather=True)
    sg, sel = sg.cpu().numpy(), sel.cpu().numpy().astype(np.int64)
    so, _ = orc.bic_select(o, x, T, T_max, N)
    assert np.all(np.abs(sg - so) <= TOL * (1 + np.abs(so)))
    # the integer decision, taken on the kernel's FP32 scores, is the oracle's rule
    np.testing.assert_array_equal(sel, orc.top_n(sg.astype(np.float64), N))
    # the gathered batch is the selected candidates' rows
    np.testing.assert_array_equal(xs.cpu().numpy(), x[sel])
    np.testing.assert_array_equal(Ts.cpu().numpy(), T[sel])
    # and valid against the FP64 scores up to the score tolerance
    if 0 < N < Bc:
        rest = np.setdiff1d(np.arange(Bc), sel)
        assert so[sel].min() >= so[rest].max() - 2 * TOL * (1 + so.max())


def test_bic_select_ties_nan_and_state_only(ctx):
    import torch
    from paper_2602_19699_amd import cbic
    x, T, T_max = I.bic_candidates("pm16k", 3000, seed=23)
    x[1000:2000] = x[:1000]  # duplicated candidates: exactly tied scores
    T[1000:2000] = T[:1000]
    x[[2500, 2600, 2700]] = np.nan  # NaN scores rank lowest
    g, o = _nets(5, 32, 2, 1, seed=9, act=1, out_act=2)
    for N in (10, 1500, 2997, 2998, 3000):
        sg, sel = cbic.bic_select(ctx, g, torch.as_tensor(x, device="cuda"), torch.as_tensor(T, device="cuda"),
                                  T_max, N)
        sg, sel = sg.cpu().numpy(), sel.cpu().numpy().astype(np.int64)
        assert np.array_equal(sg[:1000], sg[1000:2000])
        np.testing.assert_array_equal(sel, orc.top_n(sg.astype(np.float64), N))
        if N <= 2997:
            assert not {2500, 2600, 2700} & set(sel.tolist())
    # a network of the state alone (no time input)
    g2, o2 = _nets(4, 64, 1, 1, seed=3, out_act=2)
    xs = x[2000:2400]
    sg, sel = cbic.bic_select(ctx, g2, torch.as_tensor(xs, device="cuda"), None, T_max, 50)
    so, _ = orc.bic_select(o2, xs, None, T_max, 50)
    assert np.all(np.abs(sg.cpu().numpy() - so) <= TOL * (1 + np.abs(so)))
    np.testing.assert_array_equal(sel.cpu().numpy(), orc.top_n(sg.cpu().numpy().astype(np.float64), 50))


def _check_rollout(kind, p, o, x0, T_max, T, U, X, label):
    """Per step, the oracle's FP64 actor on the kernel's state gives the
    kernel's control to the network tolerance, and the kernel's next state is
    the FP64 dynamics of that state and control; zero past the horizon."""
    n = x0.shape[1]
    for b in range(len(x0)):
        Tb = T_max if T is None else int(T[b])
        if Tb < 1 or Tb > T_max:
            assert np.all(U[b] == 0) and np.all(X[b] == 0), f"{label} #{b}"
            continue
        np.testing.assert_array_equal(X[b, 0], x0[b])
        inp = np.concatenate([X[b, :Tb], ((T_max - Tb + np.arange(Tb)) / T_max)[:, None]], axis=1)
        uo = orc.mlp_forward(o, inp)
        assert np.all(np.abs(U[b, :Tb] - uo) <= TOL * (1 + np.abs(uo))), f"{label} #{b}: control"
        d, _ = orc.check_trajectory(kind, p, X[b, :Tb + 1], U[b, :Tb])
        assert d <= 1e-12, f"{label} #{b}: dynamics residual {d:.2e}"
        assert np.all(U[b, Tb:] == 0) and np.all(X[b, Tb + 1:] == 0)


@pytest.mark.parametrize("kind", [PM, P3], ids=["pm", "arm"])
def test_actor_rollout(ctx, kind):
    import torch
    from paper_2602_19699_amd import cbic
    if kind == PM:
        p, x0, T_max, scale = I.point_mass_params(0), I.point_mass_x0(300, seed=31), 100, 10.0
    else:
        p, x0, T_max, scale = I.planar3_params(0), I.planar3_x0(200, seed=32), 200, 8.0
    T = I.horizons(len(x0), 1, T_max, seed=4)
    T[[3, 7]] = [0, T_max + 1]  # outside 1..T_max: zero rows
    n, m = x0.shape[1], (2 if kind == PM else 3)
    sys_ = cbic.System(ctx, kind, p)
    for width, depth in ((32, 2), (64, 3)):
        g, o = _nets(n + 1, width, depth, m, seed=width + depth, act=0, out_act=1, scale=scale)
        U, X = cbic.actor_rollout(ctx, sys_, g, torch.as_tensor(x0, device="cuda"), T_max,
                                  T=torch.as_tensor(T, device="cuda"), states=True)
        U, X = U.cpu().numpy(), X.cpu().numpy()
        _check_rollout(kind, p, o, x0, T_max, T, U, X, f"actor {kind} w{width}")
        if kind == PM:
            # whole rollouts against the oracle's own (stable dynamics keep the
            # FP32 network differences small)
            Uo, Xo = orc.actor_rollout(kind, p, o, x0, T_max, T=T)
            assert np.all(np.abs(U - Uo) <= 1e-3 * (1 + np.abs(Uo)))
    sys_.close()


def test_bic_pipeline_feeds_the_solver(ctx):
    # select 64 of 640 candidates, roll the actor out from them, solve from that
    # warm start.  The solve is held per instance to the oracle's solve from the
    # same warm start (the actor's FP32 rollout is checked against the oracle's
    # actor in the tests above); the whole pipeline is compared with the
    # oracle's own pipeline on the candidates both pick, for the record
    import torch
    from paper_2602_19699_amd import cbic
    kind, p, _, _, _ = I.workload("pm64")
    x, T, T_max = I.bic_candidates("pm16k", 640, seed=41)
    std, std_o = _nets(5, 64, 2, 1, seed=76, act=0, out_act=2)
    g, o = _nets(5, 64, 2, 2, seed=77, act=0, out_act=1, scale=10.0)
    sys_ = cbic.System(ctx, kind, p)
    _, sel, xs, Ts = cbic.bic_select(ctx, std, torch.as_tensor(x, device="cuda"), torch.as_tensor(T, device="cuda"),
                                     T_max, 64, gather=True)
    U0 = cbic.actor_rollout(ctx, sys_, g, xs, T_max, T=Ts)
    xs, Ts, U0 = xs.cpu().numpy(), Ts.cpu().numpy(), U0.cpu().numpy()
    opt = dict(max_iter=200, stop_mode=1, rtol=1e-12)
    gs = gpu_solve(ctx, kind, p, xs, T_max, T=Ts, U0=U0, trace=True, **opt)
    sys_.close()
    oo = oracle_opts(**opt)
    r, rps = oracle_ensemble(kind, p, xs, T_max, T=Ts, U0=U0, opts=oo)
    check_parity(gs, kind, p, xs, T_max, Ts, oo, r, rps, U0=U0, label="BIC pipeline solve")
    _, sel_o = orc.bic_select(std_o, x, T, T_max, 64)
    Uo, _ = orc.actor_rollout(kind, p, o, x[sel_o], T_max, T=T[sel_o])
    ro = orc.solve_batch(kind, p, x[sel_o], T_max, T=T[sel_o], U0=Uo, opts=oo)
    sel = sel.cpu().numpy()
    both = np.intersect1d(sel, sel_o)
    assert len(both) >= 60
    e = rel(gs["J"][np.searchsorted(sel, both)], ro.J[np.searchsorted(sel_o, both)])
    print(f"BIC pipeline vs the oracle's pipeline: {len(both)} common candidates, median rel cost "
          f"{np.median(e):.2e}, max {e.max():.2e}")


def test_network_errors(ctx):
    import torch
    from paper_2602_19699_amd import cbic
    g, _ = _nets(5, 32, 1, 2, seed=1)
    kind, p, x0, T_max, _ = I.workload("pm64")
    q = I.quad_params(0)
    sq = cbic.System(ctx, QUAD, q)
    gq, _ = _nets(38, 32, 1, 12, seed=1)
    with pytest.raises(cbic.CbicError) as e:
        cbic.actor_rollout(ctx, sq, gq, torch.as_tensor(I.quad_x0(2, q), device="cuda"), 10)
    assert e.value.code == cbic.E_UNSUPPORTED
    sq.close()
    sp = cbic.System(ctx, kind, p)
    bad = cbic.Mlp(4, 32, 1, 2, g.params)  # in_dim must be n + 1 = 5
    with pytest.raises(cbic.CbicError) as e:
        cbic.actor_rollout(ctx, sp, bad, torch.as_tensor(x0, device="cuda"), T_max)
    assert e.value.code == cbic.E_INVALID
    for kw in (dict(width=48), dict(depth=5), dict(act=7), dict(out_dim=17)):
        m = cbic.Mlp(**{**dict(in_dim=5, width=32, depth=1, out_dim=2, params=g.params), **kw})
        with pytest.raises(cbic.CbicError) as e:
            m.param_count()
        assert e.value.code == cbic.E_INVALID
    assert g.param_count() == I.mlp_param_count(5, 32, 1, 2)
    with pytest.raises(cbic.CbicError) as e:  # N > Bc
        cbic.bic_select(ctx, _nets(5, 32, 1, 1, seed=2)[0], torch.zeros((10, 4), device="cuda"),
                        torch.ones(10, dtype=torch.int32, device="cuda"), 100, 11)
    assert e.value.code == cbic.E_INVALID
    sp.close()
