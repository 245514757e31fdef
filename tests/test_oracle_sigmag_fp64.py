"""Pins for the oracle's binary64 sigma_G keep decision (Section 3.1,
Eqs. 1-5 evaluated in FP64) and for its relation to the binary32 decision.

* Hand-worked lightcurves: an exact boundary in FP64, the FP64 margins of a
  worked example, and a lightcurve whose binary32 and binary64 decisions
  differ for a reason that can be followed by hand (a halfway case that
  rounds to even).
* Brute force in Python floats (``tests/bruteforce.sigmag_keep64``), for the
  standalone filter and for the exhaustive search.
* The binary32 decision differs from the binary64 one only on epochs whose
  FP64 margin lies within the binary32 rounding bound
  (``tests/parity.f32_margin_bound``), on many near-boundary lightcurves.
* Explicit grid trajectories (``oracle.eval_grid``) reproduce the search's
  result slots in both precisions.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from tests import bruteforce as bf
from tests import parity as P

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_constants.json")))
C = GOLD["sigma_g_coefficient_25_75"]["value"]


def test_exact_boundary_is_kept_in_fp64(oracle_mod):
    """With C = 0.75 and unit weights every quantity is exact: sorted
    0, 1, 2, 3, 5 gives x25 = 1, x50 = 2, x75 = 3, sigma_G = 1.5 and a
    threshold of exactly 3; the point 5 lies exactly on it and is kept
    (inclusive comparison); its successor in binary32 is dropped."""
    just_above = float(np.nextafter(np.float32(5.0), np.float32(6.0)))
    curves = np.array([[3, 0, 5, 1, 2], [3, 0, just_above, 1, 2]], np.float32)
    for d in ("f32", "f64"):
        keep, lh = oracle_mod.sigmag(curves, coeff=0.75, n_sigma=2.0, decision=d)
        assert int(keep[0]) == 0b11111, d
        assert int(keep[1]) == 0b11011, d
        assert lh[0] == pytest.approx(11.0 / math.sqrt(5.0), rel=1e-15)


def test_fp64_margins_of_worked_example(oracle_mod):
    """1, 2, 3, 4, 100: x50 = 3, threshold 2 * 0.7413 * 2 = 2.9652; the
    margins |nu - 3| - 2.9652 are -0.9652, -1.9652, -2.9652, -1.9652 and
    94.0348, and the largest |nu| is 100."""
    keep, lh, margin, numax = oracle_mod.sigmag(
        np.array([[1, 2, 3, 4, 100]], np.float32), coeff=C, decision="f64",
        want_margin=True)
    assert int(keep[0]) == 0b01111
    thr = 2.0 * C * 2.0
    want = [2 - thr, 1 - thr, 0 - thr, 1 - thr, 97 - thr]
    assert margin[0] == pytest.approx(want, abs=1e-13)
    assert numax[0] == 100.0
    assert lh[0] == pytest.approx(5.0, abs=1e-12)


def test_margins_nan_where_epoch_does_not_take_part(oracle_mod):
    ps = np.array([[1, 2, 3, 4, 100, 7]], np.float32)
    ph = np.array([[1, 1, 0, 1, 1, 1]], np.float32)        # epoch 2: phi = 0
    valid = np.array([[1, 1, 1, 1, 1, 0]], np.uint8)        # epoch 5 invalid
    _, _, margin, _ = oracle_mod.sigmag(ps, ph, valid, decision="f64",
                                        want_margin=True)
    assert np.isnan(margin[0, 2]) and np.isnan(margin[0, 5])
    assert np.all(np.isfinite(margin[0, [0, 1, 3, 4]]))


def test_binary32_and_binary64_decisions_differ_by_hand():
    """Unit weights, values -1, 0, 2^-24, 1, v with v the binary32 value just
    above fl32(1.4826) (= 1.4826000928878784): x25 = 0, x50 = 2^-24, x75 = 1.
    In FP64 the threshold is 2 * 0.7413 = 1.4826 and the distance of v is
    v - 2^-24 = 1.48260003328..., above it: v is dropped.  In binary32 the
    distance v - 2^-24 lies exactly halfway between two binary32 values and
    rounds to the even one, 1.4825999736785889, which equals the binary32
    threshold 2 * fl32(0.7413): v is kept."""
    import oracle
    oracle._load()
    v = float(np.nextafter(np.float32(1.4826), np.float32(2.0)))
    assert v == 1.4826000928878784
    curve = np.array([[-1.0, 0.0, 2.0 ** -24, 1.0, v]], np.float32)
    k32, _ = oracle.sigmag(curve, coeff=C, decision="f32")
    k64, _, margin, numax = oracle.sigmag(curve, coeff=C, decision="f64",
                                          want_margin=True)
    assert int(k32[0]) == 0b11111
    assert int(k64[0]) == 0b01111
    # the disagreement is certified: the FP64 margin is inside the bound
    assert 0.0 < margin[0, 4] <= P.f32_margin_bound(numax[0], C)
    assert margin[0, 4] == pytest.approx(v - 2.0 ** -24 - 2.0 * C, abs=1e-16)


@pytest.mark.parametrize("T", [1, 2, 3, 5, 17, 26, 60, 64])
def test_fp64_decision_matches_bruteforce(oracle_mod, T):
    rng = np.random.default_rng(500 + T)
    n = 400
    ps = rng.standard_t(3, size=(n, T)).astype(np.float32)
    ph = rng.uniform(0.05, 4.0, size=(n, T)).astype(np.float32)
    valid = (rng.random((n, T)) > 0.2).astype(np.uint8)
    ph[rng.random((n, T)) < 0.03] = 0.0
    ps[:20] = 2.5
    ph[:20] = 1.0
    keep, lh = oracle_mod.sigmag(ps, ph, valid, decision="f64")
    for c in range(n):
        idx = [i for i in range(T) if valid[c, i] and ph[c, i] > 0]
        flags = bf.sigmag_keep64([ps[c, i] for i in idx], [ph[c, i] for i in idx],
                                 0.25, 0.75, 0.7413, 2.0)
        want = sum(1 << i for i, f in zip(idx, flags) if f)
        assert int(keep[c]) == want, (c, T)
        kp = [i for i, f in zip(idx, flags) if f]
        if kp:
            sp = math.fsum(float(ps[c, i]) for i in kp)
            sf = math.fsum(float(ph[c, i]) for i in kp)
            assert lh[c] == pytest.approx(sp / math.sqrt(sf), rel=1e-13)
        else:
            assert np.isneginf(lh[c])


@pytest.mark.parametrize("quantity", [0, 1])
def test_binary32_differs_only_within_rounding_bound(oracle_mod, quantity):
    """Near-boundary lightcurves (a point placed at the FP64 threshold plus a
    few binary32 ulps either way): every epoch where the two decisions
    disagree has an FP64 margin within the binary32 rounding bound, and
    disagreements do occur (the bound is exercised, not vacuous)."""
    rng = np.random.default_rng(77 + quantity)
    n, T = 20000, 26
    ps = rng.normal(0.0, 1.0, (n, T))
    ph = rng.uniform(0.5, 2.0, (n, T)) if quantity == 0 else np.ones((n, T))
    ps32, ph32 = ps.astype(np.float32), ph.astype(np.float32)
    # move epoch 0 onto the FP64 threshold of its lightcurve, then jitter
    _, _, margin, _ = oracle_mod.sigmag(ps32, ph32, quantity=quantity, decision="f64",
                                        want_margin=True)
    scale = np.sqrt(ph32[:, 0].astype(np.float64)) if quantity == 0 else ph32[:, 0]
    nu0 = ps32[:, 0].astype(np.float64) / scale
    sgn = np.where(nu0 >= np.median(nu0), 1.0, -1.0)
    target = nu0 - sgn * margin[:, 0]            # |nu0 - x50| = thr
    ulps = rng.integers(-3, 4, n)
    val = (target * scale).astype(np.float32)
    val = np.array([np.float32(v) + np.float32(u) * np.spacing(np.float32(v))
                    for v, u in zip(val, ulps)], np.float32)
    ps32[:, 0] = val
    k32, _ = oracle_mod.sigmag(ps32, ph32, quantity=quantity, decision="f32")
    k64, _, margin, numax = oracle_mod.sigmag(ps32, ph32, quantity=quantity,
                                              decision="f64", want_margin=True)
    diff = k32 ^ k64
    bits = np.array([[(int(d) >> i) & 1 for i in range(T)] for d in diff], bool)
    assert bits.any(), "no disagreement exercised"
    bound = P.f32_margin_bound(numax)[:, None] * np.ones((1, T))
    assert np.all(np.abs(margin[bits]) <= bound[bits])
    # away from the boundary the two decisions always agree
    far = np.abs(margin) > P.f32_margin_bound(numax)[:, None]
    assert not np.any(bits & far)


@pytest.mark.parametrize("seed,sigmag,k,min_obs", [(21, 1, 3, 1), (22, 1, 1, 3),
                                                    (23, 1, 5, 2)])
def test_fp64_search_matches_bruteforce(oracle_mod, seed, sigmag, k, min_obs):
    st = synth.tiny_stack(seed, W=13, H=9, T=6, n_vel=7, mask_rate=0.1)
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    psi, phi = psi.astype(np.float32), phi.astype(np.float32)
    got = oracle_mod.search(psi, phi, st.times, st.vels, k=k, min_obs=min_obs,
                            sigmag=sigmag, decision="f64")
    ref = bf.search(psi, phi, st.times, st.vels, k, min_obs, sigmag,
                    decision="f64")
    assert np.array_equal(got["vel_idx"], ref["vel_idx"])
    assert np.array_equal(got["keep"], ref["keep"])
    fin = np.isfinite(ref["lh"])
    assert np.array_equal(np.isfinite(got["lh"]), fin)
    assert np.allclose(got["lh"][fin], ref["lh"][fin], rtol=1e-12)


@pytest.mark.parametrize("decision", ["f32", "f64"])
def test_eval_grid_reproduces_search_slots(oracle_mod, decision):
    st = synth.make_config(2, size=(90, 70), n_vel=(6, 6))
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    psi, phi = psi.astype(np.float32), phi.astype(np.float32)
    p = dict(st.params)
    p.update(k=4, min_obs=5)
    res = oracle_mod.search(psi, phi, st.times, st.vels, decision=decision, **p)
    ys, xs, ss = np.nonzero(res["vel_idx"] >= 0)
    starts = np.stack([xs, ys], 1)
    vels = st.vels[res["vel_idx"][ys, xs, ss]]
    ev = oracle_mod.eval_grid(psi, phi, st.times, starts, vels, decision=decision,
                              want_margin=True, **p)
    for key in ("lh", "flux", "lh_raw"):
        assert np.array_equal(ev[key], res[key][ys, xs, ss]), key
    assert np.array_equal(ev["keep"], res["keep"][ys, xs, ss])
    assert np.array_equal(ev["n_obs"], res["n_obs"][ys, xs, ss])
    # margins: negative exactly on the kept epochs in the FP64 decision
    if decision == "f64":
        kept = np.array([[(int(kk) >> i) & 1 for i in range(st.T)]
                         for kk in ev["keep"]], bool)
        part = np.isfinite(ev["margin"])
        assert np.array_equal(kept, part & (ev["margin"] <= 0))
    # a dropped trajectory (start far outside the image): -inf, NaN margins
    far = oracle_mod.eval_grid(psi, phi, st.times, [[-500, -500]], st.vels[:1],
                               decision=decision, want_margin=True, **p)
    assert np.isneginf(far["lh"][0]) and far["n_obs"][0] == 0
    assert np.all(np.isnan(far["margin"]))
