"""Pins of the iteration-budget calibration (paper Sec. IV-A): the
nearest-rank percentile on hand-worked lists, the linear-quadratic closed form
(one iteration reaches the optimum), and the meaning of
the budget on a point-mass batch (p99 iterations cover at least 99 % of the
instances, p50 at least half, and no smaller budget does)."""
import numpy as np
import pytest

from paper_2602_19699_amd import inputs as I

LQ, PM = I.SYS_LQ, I.SYS_POINT_MASS


@pytest.mark.parametrize("values,q,expect", [
    (list(range(1, 101)), 99, 99),   # rank ceil(99) = 99
    (list(range(1, 101)), 50, 50),
    ([3, 3, 3, 7], 50, 3),           # rank 2
    ([3, 3, 3, 7], 99, 7),           # rank ceil(3.96) = 4
    ([7, 3, 3, 3], 99, 7),           # order does not matter
    ([5], 99, 5),
    ([1, 2], 50, 1),                 # rank 1
    ([1, 2], 99, 2),
    (list(range(1, 201)), 99, 198),  # rank 198
])
def test_nearest_rank_hand_worked(orc, values, q, expect):
    assert orc.percentile_nearest_rank(values, q) == expect


def test_lq_all_progress_in_the_first_iteration(orc):
    # linear dynamics, quadratic cost: the first Newton step is the optimum;
    # a second iteration can only move the cost by rounding (then it is
    # accepted and the tolerance stop ends the solve) or not at all (then the
    # line search fails), so every count is 1 or 2 and the cost after the
    # first iteration is final
    for n, m in [(2, 1), (4, 2), (6, 3)]:
        p = I.lq_random(n, m, seed=n)
        x0 = I.lq_x0(16, n)
        p99, p50, counts = orc.calibrate_max_iter(LQ, p, x0, 12, cap=1000)
        assert set(counts.tolist()) <= {1, 2} and 1 <= p50 <= p99 <= 2
        r = orc.solve_batch(LQ, p, x0, 12, opts=orc.Options(max_iter=1000, stop_mode=1))
        first = r.trace[:, 1]
        assert np.all(np.abs(r.J - first) <= 1e-12 * np.abs(first))


def test_point_mass_budget_meaning(orc):
    kind, p, x0, T, _ = I.workload("pm64")
    p99, p50, counts = orc.calibrate_max_iter(kind, p, x0, T, cap=1000)
    n = len(counts)
    assert 1 <= p50 <= p99 < 1000
    assert np.sum(counts <= p99) >= 0.99 * n and np.sum(counts <= p99 - 1) < 0.99 * n
    assert np.sum(counts <= p50) >= 0.5 * n and np.sum(counts <= p50 - 1) < 0.5 * n
    # the counts are those of a plain tolerance-stop solve with the same cap
    r = orc.solve_batch(kind, p, x0, T, opts=orc.Options(max_iter=1000, stop_mode=1))
    assert np.array_equal(counts, r.iters)
