"""Pins for the oracle's sigma_G filter (Section 3.1, Eqs. 1-5).

Hand-worked lightcurves, the coefficient from erfinv, the statistical
meaning of sigma_G, and invariances.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special

from tests import bruteforce as bf

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_constants.json")))
C = GOLD["sigma_g_coefficient_25_75"]["value"]
NS = GOLD["sigma_g_example_n"]["value"]


def test_coefficient_from_erfinv():
    """Eq. 3-5: sigma_G = (x75 - x25) / (sqrt2 (erfinv(0.5) - erfinv(-0.5))).
    The printed 0.7413 agrees to 2e-6.  Eq. 4 as printed omits the sqrt(2)
    of Eq. 3; without it the coefficient would be 1.048, not 0.7413."""
    exact = 1.0 / (math.sqrt(2.0) * (special.erfinv(0.5) - special.erfinv(-0.5)))
    assert abs(exact - C) < 2e-6
    garbled = 1.0 / (special.erfinv(0.5) - special.erfinv(-0.5))
    assert abs(garbled - 1.0483) < 1e-3


def test_sigma_g_estimates_gaussian_sigma():
    """The estimator itself: 0.7413 * IQR of many N(0, s^2) draws ~ s."""
    rng = np.random.default_rng(11)
    s = 3.7
    x = rng.normal(0.0, s, size=1_000_000)
    q25, q75 = np.percentile(x, [25, 75])
    assert abs(C * (q75 - q25) / s - 1.0) < 5e-3


def test_hand_worked_outlier(oracle_mod):
    # values 1,2,3,4,100 (unit weights): ranks 1,2,3 -> x25=2, x50=3, x75=4,
    # sigma = 0.7413*2, thr = 2.9652: 1..4 kept, 100 dropped,
    # L' = (1+2+3+4)/sqrt(4) = 5.
    keep, lh = oracle_mod.sigmag(np.array([[1, 2, 3, 4, 100]], np.float32),
                                 coeff=C, n_sigma=NS)
    assert int(keep[0]) == 0b01111
    assert lh[0] == pytest.approx(5.0, abs=1e-12)


def test_hand_worked_low_outlier(oracle_mod):
    # sorted -50,1,2,3,4: x25=1, x50=2, x75=3, thr=2.9652; -50 is dropped
    keep, lh = oracle_mod.sigmag(np.array([[3, -50, 1, 4, 2]], np.float32))
    assert int(keep[0]) == 0b11101
    assert lh[0] == pytest.approx(10.0 / 2.0, abs=1e-12)


def test_constant_lightcurve_keeps_everything(oracle_mod):
    """IQR = 0 gives a zero threshold; the inclusive comparison keeps every
    point (a strict comparison would drop them all)."""
    for T in (1, 2, 5, 26, 64):
        keep, lh = oracle_mod.sigmag(np.full((1, T), 7.5, np.float32))
        assert int(keep[0]) == (1 << T) - 1
        assert lh[0] == pytest.approx(7.5 * T / math.sqrt(T), rel=1e-14)


def test_t1_and_t2(oracle_mod):
    keep, lh = oracle_mod.sigmag(np.array([[4.0]], np.float32))
    assert int(keep[0]) == 1 and lh[0] == 4.0
    # T=2: x25 = s[0], x50 = x75 = s[1]; thr = 1.4826 (b - a) >= b - a
    keep, lh = oracle_mod.sigmag(np.array([[1.0, 9.0]], np.float32))
    assert int(keep[0]) == 3


def test_ties_at_quantiles(oracle_mod):
    # T=5 with ties: sorted 2,2,2,2,9 -> x25=x50=x75=2, thr=0 -> 9 dropped
    keep, _ = oracle_mod.sigmag(np.array([[2, 9, 2, 2, 2]], np.float32))
    assert int(keep[0]) == 0b11101


def test_quantile_ranks_nearest_rank():
    """Nearest-rank selection index floor(q (n-1) + 1/2): T=26 -> 6, 13, 19."""
    def r(q, n):
        return int(math.floor(q * (n - 1) + 0.5))
    assert [r(q, 26) for q in (0.25, 0.5, 0.75)] == [6, 13, 19]
    assert [r(q, 5) for q in (0.25, 0.5, 0.75)] == [1, 2, 3]
    assert [r(q, 60) for q in (0.25, 0.5, 0.75)] == [15, 30, 44]


def test_invalid_epochs_are_ignored(oracle_mod):
    rng = np.random.default_rng(3)
    base = rng.normal(size=(200, 17)).astype(np.float32)
    ph = rng.uniform(0.5, 2.0, size=base.shape).astype(np.float32)
    valid = (rng.random(base.shape) > 0.2).astype(np.uint8)
    junk = base.copy()
    junk[valid == 0] = 1e6            # would dominate every quantile
    k1, l1 = oracle_mod.sigmag(base, ph, valid)
    k2, l2 = oracle_mod.sigmag(junk, ph, valid)
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_array_equal(l1, l2)
    bits = np.array([[int(k) >> i & 1 for i in range(17)] for k in k1])
    assert not np.any(bits[valid == 0])
    # phi <= 0 also removes the epoch
    ph2 = ph.copy()
    ph2[valid == 0] = 0.0
    k3, l3 = oracle_mod.sigmag(junk, ph2, None)
    np.testing.assert_array_equal(k1, k3)


def test_matches_bruteforce(oracle_mod):
    rng = np.random.default_rng(5)
    for T in (1, 2, 3, 7, 26, 40, 64):
        ps = rng.standard_t(3, size=(50, T)).astype(np.float32)
        ph = rng.uniform(0.2, 3.0, size=(50, T)).astype(np.float32)
        keep, lh = oracle_mod.sigmag(ps, ph)
        for c in range(50):
            kf = bf.sigmag_keep(ps[c], ph[c], 0.25, 0.75, C, NS)
            kb = sum(1 << i for i, k in enumerate(kf) if k)
            assert int(keep[c]) == kb
            sp = math.fsum(float(ps[c, i]) for i in range(T) if kf[i])
            sf = math.fsum(float(ph[c, i]) for i in range(T) if kf[i])
            assert lh[c] == pytest.approx(sp / math.sqrt(sf), rel=1e-13)


def test_scale_and_permutation_invariance(oracle_mod):
    rng = np.random.default_rng(6)
    ps = rng.normal(size=(300, 26)).astype(np.float32)
    ph = rng.uniform(0.2, 3.0, size=ps.shape).astype(np.float32)
    k1, l1 = oracle_mod.sigmag(ps, ph)
    # psi -> 2 psi, phi -> 4 phi leaves nu_i bit-identical
    k2, l2 = oracle_mod.sigmag(ps * 2, ph * 4)
    np.testing.assert_array_equal(k1, k2)
    np.testing.assert_allclose(l1, l2, rtol=1e-14)
    perm = rng.permutation(26)
    k3, l3 = oracle_mod.sigmag(ps[:, perm], ph[:, perm])
    bits1 = np.array([[int(k) >> i & 1 for i in range(26)] for k in k1])
    bits3 = np.array([[int(k) >> i & 1 for i in range(26)] for k in k3])
    np.testing.assert_array_equal(bits1[:, perm], bits3)
    np.testing.assert_allclose(l1, l3, rtol=1e-13)


def test_gaussian_keep_fraction(oracle_mod):
    """For Gaussian lightcurves 2 sigma_G ~ 2 sigma, so about 95% of points
    survive (finite-sample quantile noise lowers it slightly)."""
    rng = np.random.default_rng(7)
    ps = rng.normal(size=(20000, 60)).astype(np.float32)
    keep, _ = oracle_mod.sigmag(ps)
    frac = np.mean([bin(int(k)).count("1") for k in keep]) / 60
    assert 0.93 < frac < 0.97
