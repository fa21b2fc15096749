"""The algorithmic byte and flop counts behind the roofline figures of
bench.py, against counts written out by hand for small cases (host only)."""
import numpy as np

import bench


def test_iteration_bytes_by_hand():
    # point mass (n=4, m=2, FP32): instance 0 swept twice and read 250 rollout
    # steps, writing 120; instance 1 swept once, read 100, wrote 100
    work = np.array([[2, 3, 250, 120], [1, 1, 100, 100]], np.int32)
    Tb = np.array([100, 60])
    per_step = 4 + 2 + 8 + 2  # x, u, K, k
    words = 2 * (100 * per_step + 4) + 250 * per_step + 120 * 6 + 1 * (60 * per_step + 4) + 100 * per_step + 100 * 6
    assert bench.alg_bytes(work, Tb, 4, 2, 4) == words * 4


def test_finalisation_bytes_by_hand():
    # two instances of horizons 3 and 5 in a batch of T_max = 5 (n=4, m=2, FP32
    # workspace): the final trajectories read once, every output row written
    reads = ((3 + 1) * 4 + 3 * 2 + (5 + 1) * 4 + 5 * 2) * 4
    rows = 6 * 4 + 5 * 2 + 6 * (1 + 2 * 4)  # X, U, then V-bar, V_x, x_{k+K}
    assert bench.final_bytes([3, 5], 5, 4, 2, 4) == reads + 2 * (rows * 8 + 32)
    assert bench.final_bytes([3, 5], 5, 4, 2, 4, targets=False) == reads + 2 * ((6 * 4 + 5 * 2) * 8 + 32)

