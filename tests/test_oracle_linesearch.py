"""Pins of the oracle's line search, its Levenberg-Marquardt schedule of mu,
its replay of given step indices and its FP32-storage probe, on the point
mass, whose linear dynamics make one iLQR iteration a Newton step of the dense
model built independently in pm_dense (numpy, no Riccati recursion).

Line search (reading of Sec. IV-B, which names the search but not its rule):
the trials alpha = beta^j, j = 0, 1, ..., and the FIRST one whose cost is
finite and strictly below J is taken, not the best one.  The closed-loop
rollout of a linear system with step alpha moves the controls by exactly
alpha d, d the Newton step, so every trial cost is J(U + alpha d).

Levenberg-Marquardt (Sec. IV-B): without the eigenvalue clip the model
Hessian H may be indefinite; an iteration starts from the current mu, raises
it by the factor while H + mu I does not factorise or no trial lowers J,
takes the step -(H + mu I)^-1 g, then lowers mu by the factor (not below
mu0) for the next iteration."""
import dataclasses

import numpy as np

from paper_2602_19699_amd import inputs as I

from pm_dense import cost, dense_model

PM = I.SYS_POINT_MASS
T = 60


def _clip(orc):
    return lambda M: orc.psd_clip(0.5 * (M + M.T), 1e-6)


def _newton_step(orc, p, x0, U):
    g, H = dense_model(orc, p, x0, U, _clip(orc))
    return -np.linalg.solve(H, g).reshape(U.shape)


def _case(b, w_obs=5.0):
    p = I.point_mass_params(0, w_obs=w_obs)
    return p, I.point_mass_x0(200, 7)[b]


def test_first_accepted_trial_is_taken_not_the_best(orc):
    p, x0 = _case(0)
    U0 = np.zeros((T, 2))
    d = _newton_step(orc, p, x0, U0)
    J0, J1, Jh = cost(orc, p, x0, U0), cost(orc, p, x0, U0 + d), cost(orc, p, x0, U0 + 0.5 * d)
    # the full step lowers J, the half step would lower it further
    assert J1 < J0 and Jh < J1 - 10.0
    r = orc.solve_batch(PM, p, x0[None], T, opts=orc.Options(max_iter=1))
    assert r.jtrace[0, 0] == 0 and r.iters[0] == 1
    np.testing.assert_allclose(r.U[0], U0 + d, atol=1e-9 * np.abs(d).max(), rtol=0)
    assert abs(r.J[0] - J1) <= 1e-12 * J1


def test_full_step_rejected_half_step_taken(orc):
    p, x0 = _case(44)
    U0 = np.zeros((T, 2))
    d = _newton_step(orc, p, x0, U0)
    J0, J1, Jh = cost(orc, p, x0, U0), cost(orc, p, x0, U0 + d), cost(orc, p, x0, U0 + 0.5 * d)
    assert J1 >= J0 and Jh < J0
    r = orc.solve_batch(PM, p, x0[None], T, opts=orc.Options(max_iter=1))
    assert r.jtrace[0, 0] == 1
    np.testing.assert_allclose(r.U[0], U0 + 0.5 * d, atol=1e-9 * np.abs(d).max(), rtol=0)
    assert abs(r.J[0] - Jh) <= 1e-12 * Jh
    # the closest call among the tried trials: the rejected full step
    assert np.isclose(r.margin[0, 0], min(abs(J1 - J0), abs(Jh - J0)) / J0, rtol=1e-9)


def _lm_reference(orc, p, x0, U, iters, mu0=1e-6, fac=10.0, beta=0.5, trials=16):
    """The Levenberg-Marquardt schedule on the dense model: returns each
    iteration's accepted mu, controls and the condition number of H + mu I.  Every mu it tries is kept away from
    the factorisation boundary (smallest eigenvalue of H + mu I not within
    1e-6 of 0 relative to |H|), so the oracle's Cholesky decides alike."""
    sym = lambda M: 0.5 * (M + M.T)
    mu, out = mu0, []
    J = cost(orc, p, x0, U)
    for _ in range(iters):
        g, H = dense_model(orc, p, x0, U, sym)
        nh = np.abs(np.linalg.eigvalsh(H)).max()
        while True:
            lmin = np.linalg.eigvalsh(H + mu * np.eye(len(g))).min()
            assert abs(lmin) > 1e-6 * nh, "a tried mu sits on the factorisation boundary"
            if lmin <= 0:
                mu *= fac
                continue
            d = -np.linalg.solve(H + mu * np.eye(len(g)), g).reshape(U.shape)
            a, acc = 1.0, None
            for _ in range(trials):
                Jt = cost(orc, p, x0, U + a * d)
                if np.isfinite(Jt) and Jt < J:
                    acc = a
                    break
                a *= beta
            if acc is None:
                mu *= fac
                continue
            break
        U = U + acc * d
        J = cost(orc, p, x0, U)
        out.append((mu, U, np.linalg.cond(H + mu * np.eye(len(g)))))
        mu = max(mu / fac, mu0)
    return out


def test_lm_mu_climbs_and_falls(orc):
    # obstacles of weight 20 make the model indefinite near the start: mu
    # climbs from 1e-6 to 1 in the first iteration, starts the second at 0.1
    # and climbs back to 1, then falls by the factor in every later iteration;
    # each iteration lowers J by at least 1e-4 relative, far from any near-tie
    lm = orc.Options(reg=1, eps=-np.inf, mu0=1e-6, mu_factor=10.0, mu_max=1e10)
    Tm = 40
    for b in (5, 11):
        p, x0 = _case(b, w_obs=20.0)
        ref = _lm_reference(orc, p, x0, np.zeros((Tm, 2)), 5)
        mus = [m for m, _, _ in ref]
        assert mus[0] >= 1.0 and mus[1] == mus[0], mus  # climb, and a climb back
        assert any(mus[i + 1] < mus[i] for i in range(len(mus) - 1)), mus  # a fall
        Js = [cost(orc, p, x0, np.zeros((Tm, 2)))] + [cost(orc, p, x0, U) for _, U, _ in ref]
        assert all(Js[i] - Js[i + 1] >= 1e-4 * Js[i] for i in range(len(ref)))
        for it, (mu, U, cond) in enumerate(ref, start=1):
            r = orc.solve_batch(PM, p, x0[None], Tm, opts=dataclasses.replace(lm, max_iter=it))
            assert r.iters[0] == it
            # two FP64 solves of H + mu I (block elimination and LAPACK) agree to
            # about the condition number times the rounding unit
            tol = max(1e-13 * cond, 1e-11) * max(np.abs(U).max(), 1.0)
            np.testing.assert_allclose(r.U[0], U, atol=tol, rtol=0,
                                       err_msg=f"instance {b}, iteration {it}, mu {mu:g}, cond {cond:.1e}")


def test_forced_step_indices(orc):
    # replaying the oracle's own accepted indices reproduces it bit for bit;
    # forcing another index takes that trial whatever its cost (finite only)
    p, x0 = _case(0)
    o = orc.Options(max_iter=8)
    r = orc.solve_batch(PM, p, x0[None], T, opts=o)
    rr = orc.solve_batch(PM, p, x0[None], T, opts=o, force_j=r.jtrace)
    for f in ("X", "U", "J", "iters", "status", "trace"):
        np.testing.assert_array_equal(getattr(r, f), getattr(rr, f), err_msg=f)
    U0 = np.zeros((T, 2))
    d = _newton_step(orc, p, x0, U0)
    for j in (1, 3):
        fj = np.full((1, 1), j, np.int32)
        rf = orc.solve_batch(PM, p, x0[None], T, opts=orc.Options(max_iter=1), force_j=fj)
        np.testing.assert_allclose(rf.U[0], U0 + 0.5 ** j * d, atol=1e-9 * np.abs(d).max(), rtol=0)
    # a forced "no step" (-1) freezes the instance as a failed line search
    rn = orc.solve_batch(PM, p, x0[None], T, opts=orc.Options(max_iter=1), force_j=np.full((1, 1), -1, np.int32))
    assert rn.status[0] == orc.ST_LS_FAILED and np.all(rn.U == 0)


def test_fp32_storage_probe(orc):
    # the probe keeps what the mixed form stores in FP32 representable in FP32
    # and stays near the FP64 solve on this well-conditioned workload
    kind, p, x0, Tm, _ = I.workload("pm64")
    r = orc.solve_batch(kind, p, x0, Tm, opts=orc.Options(max_iter=20))
    q = orc.solve_batch(kind, p, x0, Tm, opts=orc.Options(max_iter=20, round32=1))
    for a in (q.X, q.U):
        np.testing.assert_array_equal(a, a.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(q.J - r.J) <= 1e-4 * np.abs(r.J))
    assert np.any(q.J != r.J)
