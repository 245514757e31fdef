"""Pins for the sigma_G variants of Section 3.1: the filtered quantity
(likelihood psi/sqrt(phi) or flux psi/phi) and the constant C of Eq. 3 for
user-chosen quantile pairs."""
import math

import numpy as np
import pytest
from scipy import stats

F32 = np.float32


def _bf_keep(ps, ph, quantity, q_lo, q_hi, coeff, n_sigma):
    vals = [F32(a) / (F32(b) if quantity else np.sqrt(F32(b))) for a, b in zip(ps, ph)]
    s = sorted(vals)
    n = len(s)
    q = lambda qq: s[int(math.floor(qq * (n - 1) + 0.5))]
    lo, md, hi = q(q_lo), q(0.5), q(q_hi)
    thr = F32(n_sigma) * (F32(coeff) * F32(hi - lo))
    return [bool(abs(F32(v - md)) <= thr) for v in vals]


@pytest.mark.parametrize("quantity", [0, 1])
@pytest.mark.parametrize("ql,qh", [(0.25, 0.75), (0.1, 0.9)])
def test_filter_quantity_bruteforce(oracle_mod, quantity, ql, qh):
    rng = np.random.default_rng(81 + quantity)
    n, T = 300, 17
    ps = rng.normal(0, 3, (n, T)).astype(np.float32)
    ps[:, 3] += rng.choice([0, 40], n).astype(np.float32)
    ph = rng.uniform(0.2, 5, (n, T)).astype(np.float32)
    c = oracle_mod.sigmag_coeff(ql, qh)
    keep, lh = oracle_mod.sigmag(ps, ph, q_lo=ql, q_hi=qh, coeff=c, n_sigma=2.0,
                                 quantity=quantity)
    for j in range(n):
        kf = _bf_keep(ps[j], ph[j], quantity, ql, qh, c, 2.0)
        assert int(keep[j]) == sum(1 << i for i, k in enumerate(kf) if k)
        sp = math.fsum(float(a) for a, k in zip(ps[j], kf) if k)
        sf = math.fsum(float(b) for b, k in zip(ph[j], kf) if k)
        assert lh[j] == pytest.approx(sp / math.sqrt(sf), rel=1e-12)


def test_flux_equals_likelihood_for_constant_phi(oracle_mod):
    """With phi = 4 in every epoch, psi/phi = (psi/sqrt(phi)) / 2 exactly, so
    the two quantities flag the same epochs."""
    rng = np.random.default_rng(83)
    ps = rng.normal(0, 2, (500, 26)).astype(np.float32)
    ps[:, ::7] *= 9
    ph = np.full_like(ps, 4.0)
    k0, _ = oracle_mod.sigmag(ps, ph, quantity=0)
    k1, _ = oracle_mod.sigmag(ps, ph, quantity=1)
    assert np.array_equal(k0, k1)


def test_flux_and_likelihood_differ_with_varying_phi(oracle_mod):
    """Worked example, n = 8, nearest ranks 2, 4, 5 (0-based).
    psi = 1..7 with phi = 1, and psi = 0.4 with phi = 0.01 in the last epoch:
    likelihoods 1..7 and 4 -> sorted 1 2 3 4 4 5 6 7, x25 = 3, median 4,
    x75 = 5, thr = 2 * 0.7413 * 2 = 2.965: epochs with 1 and 7 dropped.
    fluxes 1..7 and 40 -> sorted 1 .. 7 40, x25 = 3, median 5, x75 = 6,
    thr = 2 * 0.7413 * 3 = 4.448: only the flux 40 dropped."""
    ps = np.array([[1, 2, 3, 4, 5, 6, 7, 0.4]], np.float32)
    ph = np.array([[1, 1, 1, 1, 1, 1, 1, 0.01]], np.float32)
    k0, _ = oracle_mod.sigmag(ps, ph, quantity=0)
    k1, _ = oracle_mod.sigmag(ps, ph, quantity=1)
    assert int(k0[0]) == 0b10111110
    assert int(k1[0]) == 0b01111111


@pytest.mark.parametrize("ql,qh", [(0.25, 0.75), (0.1, 0.9), (0.16, 0.84), (0.05, 0.6)])
def test_coeff_from_normal_quantiles(oracle_mod, ql, qh):
    c = oracle_mod.sigmag_coeff(ql, qh)
    assert c == pytest.approx(1.0 / (stats.norm.ppf(qh) - stats.norm.ppf(ql)), rel=1e-12)
    x = np.random.default_rng(84).normal(0, 3.0, 10 ** 6)
    est = c * (np.quantile(x, qh) - np.quantile(x, ql))
    assert est == pytest.approx(3.0, rel=5e-3)


def test_coeff_matches_the_printed_constant(oracle_mod):
    assert abs(oracle_mod.sigmag_coeff(0.25, 0.75) - 0.7413) < 2e-6
