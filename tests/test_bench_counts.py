"""The benchmark's own arithmetic: the lower bound on selection comparisons
behind the ALU roofline, and the exact valid-trajectory fraction reported
beside the nominal count.  CPU only."""
import math

import numpy as np
import pytest

import bench


# Minimum worst-case comparisons to find the median of n values, known
# exactly for small n (Knuth, TAOCP vol. 3, Section 5.3.3): M(3) = 3,
# M(5) = 6, M(7) = 10, M(9) = 14.
KNOWN_MEDIAN = {3: 3, 5: 6, 7: 10, 9: 14}


@pytest.mark.parametrize("n", sorted(KNOWN_MEDIAN))
def test_lower_bound_never_exceeds_known_median_cost(n):
    lb = bench.select_lower_bound(n, [(n - 1) // 2])
    assert lb <= KNOWN_MEDIAN[n]
    if n <= 5:                                   # the bound is tight there
        assert lb == KNOWN_MEDIAN[n]


@pytest.mark.parametrize("n", [2, 5, 26, 64])
def test_lower_bound_extremes(n):
    # the maximum needs exactly n - 1 comparisons
    assert bench.select_lower_bound(n, [n - 1]) == n - 1
    # the second largest needs n - 2 + ceil(log2 n) (Kislitsyn); the
    # adversary bound may not exceed it
    assert bench.select_lower_bound(n, [n - 2]) <= n - 2 + math.ceil(math.log2(n))


def test_benchmark_op_count_at_26_epochs():
    # nearest ranks of 1/4, 1/2, 3/4 for 26 values: 6, 13, 19 (0-based);
    # the median rank dominates: 25 + min(13, 12) = 37 comparisons
    assert bench.select_lower_bound(26, [6, 13, 19]) == 37
    assert bench.search_alg_ops(26, True) == pytest.approx(37 / 26 + 4)
    assert bench.search_alg_ops(26, False) == 2.0


def _valid_bruteforce(times, vels, W, H, min_obs):
    t = np.asarray(times, np.float64)
    t = t - t.min()
    v = np.asarray(vels, np.float32).astype(np.float64)
    ys, xs = np.mgrid[0:H, 0:W]
    n = 0
    for j in range(v.shape[0]):
        c = np.zeros((H, W), np.int64)
        for ti in t:
            dx, dy = np.floor(v[j, 0] * ti + 0.5), np.floor(v[j, 1] * ti + 0.5)
            c += (xs + dx >= 0) & (xs + dx < W) & (ys + dy >= 0) & (ys + dy < H)
        n += int(np.sum(c >= min_obs))
    return n


@pytest.mark.parametrize("seed,min_obs", [(0, 1), (1, 4), (2, 7), (3, 9)])
def test_valid_fraction_matches_bruteforce(seed, min_obs):
    rng = np.random.default_rng(seed)
    T, W, H = 9, 37, 23
    times = np.sort(rng.uniform(0, 2, T))
    vels = rng.uniform(-25, 25, size=(30, 2)).astype(np.float32)
    want = _valid_bruteforce(times, vels, W, H, min_obs) / (W * H * len(vels))
    assert bench.valid_fraction(times, vels, W, H, min_obs) == pytest.approx(want, abs=1e-12)
