"""Serving: continuous batching of mixed requests.  Each result is the same
alone and in the mix, served results match the batched solver and the
oracle, and admission never exceeds the memory cap."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2602_19699_amd import inputs as I

from gpu_helpers import gpu_solve, oracle_opts, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2602_19699_amd import cbic
    assert torch.cuda.is_available()
    c = cbic.Context(0)
    yield c
    c.close()


def test_alone_equals_mix_and_matches_batch_and_oracle(ctx):
    from paper_2602_19699_amd import cbic, loadgen
    mix = loadgen.Mix(ctx)
    reqs = mix.requests(48, seed=3, t_range=(10, 60))
    srv = cbic.Server(ctx, slots_per_class=64, t_max=60, iters_per_launch=3)
    tickets = [srv.submit(mix.systems[k], x0, T, opts=mix.opts) for k, T, x0 in reqs]
    srv.drain()
    res = [srv.poll(t) for t in tickets]
    st = srv.stats()
    assert st["completed"] == 48 and st["classes"] == 3 and st["max_resident"] > 1
    # the same requests alone, one at a time
    for i in (0, 5, 11, 23, 47):
        k, T, x0 = reqs[i]
        t = srv.submit(mix.systems[k], x0, T, opts=mix.opts)
        srv.drain()
        a = srv.poll(t)
        assert a["J"] == res[i]["J"] and a["iters"] == res[i]["iters"] and a["status"] == res[i]["status"]
        np.testing.assert_array_equal(a["X"], res[i]["X"])
        np.testing.assert_array_equal(a["Vbar"], res[i]["Vbar"])
    srv.close()
    # served results equal the batched solver and, for the well-conditioned
    # classes, the oracle
    for kind in (I.SYS_POINT_MASS, I.SYS_QUAD_SYNTH, I.SYS_PLANAR3):
        idx = [i for i, (k, _, _) in enumerate(reqs) if k == kind]
        if not idx:
            continue
        x0 = np.stack([reqs[i][2] for i in idx])
        T = np.array([reqs[i][1] for i in idx], np.int32)
        g = gpu_solve(ctx, kind, mix.params[kind], x0, 60, T=T, stop_mode=1, rtol=1e-10)
        for j, i in enumerate(idx):
            assert g["J"][j] == res[i]["J"]
            np.testing.assert_array_equal(g["X"][j, : T[j] + 1], res[i]["X"])
        if kind != I.SYS_PLANAR3:
            r = orc.solve_batch(kind, mix.params[kind], x0, 60, T=T, opts=oracle_opts(stop_mode=1, rtol=1e-10))
            assert np.all(rel(g["J"], r.J) <= 1e-9)


def test_admission_respects_the_memory_cap(ctx):
    # the device memory of all pools together stays within the cap: with a
    # generous cap every class gets its pool; with a cap below two one-slot
    # pools one class runs at a time, and idle pools are released for the
    # classes waiting (evictions); every request completes either way, with
    # the batched solver's result
    from paper_2602_19699_amd import cbic, loadgen
    mix = loadgen.Mix(ctx)
    reqs = mix.requests(40, seed=5, t_range=(20, 40))
    one = max(mix.systems[k].workspace_size(1, 40) for k in mix.kinds)
    for cap, expect_evictions in ((48 << 20, False), (int(1.2 * one), True)):
        srv = cbic.Server(ctx, mem_cap=cap, slots_per_class=16, t_max=40, iters_per_launch=2)
        tickets = [srv.submit(mix.systems[k], x0, T, opts=mix.opts) for k, T, x0 in reqs]
        srv.drain()
        res = [srv.poll(t, targets=False) for t in tickets]
        st = srv.stats()
        print(f"cap {cap} B: {st}")
        assert st["completed"] == 40 and st["peak_pool_bytes"] <= cap
        assert st["inflight_bytes"] == 0 and st["peak_inflight_bytes"] <= st["peak_pool_bytes"]
        assert (st["evictions"] > 0) == expect_evictions
        for kind in mix.kinds:
            idx = [i for i, (k, _, _) in enumerate(reqs) if k == kind]
            x0 = np.stack([reqs[i][2] for i in idx])
            T = np.array([reqs[i][1] for i in idx], np.int32)
            g = gpu_solve(ctx, kind, mix.params[kind], x0, 40, T=T, stop_mode=1, rtol=1e-10)
            for j, i in enumerate(idx):
                assert g["J"][j] == res[i]["J"]
        srv.close()
    # a request that can never fit is refused
    tiny = cbic.Server(ctx, mem_cap=4096, slots_per_class=4, t_max=200)
    with pytest.raises(cbic.CbicError) as e:
        tiny.submit(mix.systems[I.SYS_QUAD_SYNTH], mix.x0(I.SYS_QUAD_SYNTH, 1, 1)[0], 200, opts=mix.opts)
    assert e.value.code == cbic.E_BUSY
    tiny.close()


def test_requests_are_served_with_their_own_options(ctx):
    # requests of one system and precision with different result-affecting
    # options (budget, stop rule, control bound, Levenberg-Marquardt; lane and
    # workgroup schedules) form
    # classes of their own: each result is the batched solver's under that
    # request's options, bit for bit
    from paper_2602_19699_amd import cbic
    p = I.point_mass_params(0)
    pa = I.planar3_params(0)
    pq = I.quad_params(0)
    sp, sa = cbic.System(ctx, I.SYS_POINT_MASS, p), cbic.System(ctx, I.SYS_PLANAR3, pa)
    sq = cbic.System(ctx, I.SYS_QUAD_SYNTH, pq)
    x0, xa, xq = I.point_mass_x0(12, 4), I.planar3_x0(12, 5), I.quad_x0(12, pq, seed=6)
    variants = [dict(max_iter=7), dict(max_iter=30, stop_mode=1, rtol=1e-9), dict(max_iter=20, u_max=6.0),
                dict(max_iter=20, regularization=1), dict(max_iter=15, precision=1, u_max=6.0)]
    srv = cbic.Server(ctx, slots_per_class=32, t_max=80, iters_per_launch=3)
    jobs = []
    for vi, v in enumerate(variants):
        for sysm, kind, xs, T in ((sp, I.SYS_POINT_MASS, x0, 60), (sa, I.SYS_PLANAR3, xa, 70),
                                  (sq, I.SYS_QUAD_SYNTH, xq, 30)):
            for b in range(0, 12, 3):
                jobs.append((vi, kind, b, T, srv.submit(sysm, xs[b], T, opts=cbic.Options(**v))))
    srv.drain()
    st = srv.stats()
    assert st["classes"] == 3 * len(variants)
    for vi, v in enumerate(variants):
        for kind, xs, T, prm in ((I.SYS_POINT_MASS, x0, 60, p), (I.SYS_PLANAR3, xa, 70, pa),
                                 (I.SYS_QUAD_SYNTH, xq, 30, pq)):
            g = gpu_solve(ctx, kind, prm, xs, T, **v)
            for vj, k, b, T2, t in jobs:
                if vj == vi and k == kind:
                    r = srv.poll(t)
                    assert r["J"] == g["J"][b] and r["status"] == g["status"][b], (v, kind, b)
                    np.testing.assert_array_equal(r["U"], g["U"][b, :T2])
    srv.close()
    sp.close()
    sa.close()
    sq.close()


def test_invalid_requests_are_refused_and_the_server_keeps_serving(ctx):
    from paper_2602_19699_amd import cbic
    p = I.point_mass_params(0)
    sysm = cbic.System(ctx, I.SYS_POINT_MASS, p)
    x0 = I.point_mass_x0(2, 6)
    srv = cbic.Server(ctx, slots_per_class=8, t_max=50)
    for bad in (dict(group_lanes=3), dict(ls_beta=1.5), dict(psd_eps=float("nan")), dict(max_iter=-1),
                dict(schedule=7), dict(u_max=0.0)):
        with pytest.raises(cbic.CbicError) as e:
            srv.submit(sysm, x0[0], 30, opts=cbic.Options(**bad))
        assert e.value.code == cbic.E_INVALID, bad
    # an LQ system built for another clipping floor
    lq = cbic.System(ctx, I.SYS_LQ, I.lq_random(2, 1, seed=1))
    with pytest.raises(cbic.CbicError) as e:
        srv.submit(lq, np.ones(2), 10, opts=cbic.Options(psd_eps=1e-3))
    assert e.value.code == cbic.E_INVALID
    t = srv.submit(sysm, x0[1], 30, opts=cbic.Options(max_iter=10))
    srv.drain()
    r = srv.poll(t)
    g = gpu_solve(ctx, I.SYS_POINT_MASS, p, x0[1:], 30, max_iter=10)
    assert r["J"] == g["J"][0]
    srv.close()
    for s_ in (sysm, lq):
        s_.close()


def test_poisson_run_reports_latency(ctx):
    from paper_2602_19699_amd import cbic, loadgen
    mix = loadgen.Mix(ctx)
    srv = cbic.Server(ctx, slots_per_class=512, t_max=200, iters_per_launch=4)
    stats, res, reqs = loadgen.run_poisson(srv, mix, rate=2000.0, n=400, seed=9)
    print("poisson 2k/s:", stats)
    assert stats["p50_ms"] > 0 and stats["p99_ms"] >= stats["p50_ms"]
    assert all(r["status"] in (1, 2, 4) for r in res)
    srv.close()
