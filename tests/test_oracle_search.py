"""Pins for the oracle's trajectory search (Section 3, Sections 3.1-3.2).

Brute force on tiny stacks (every candidate of a pixel sorted, not a running
top-K), the closed form of a noise-free pixel-centred source, translation,
scaling and epoch-permutation invariances, and the N(0,1) statistics of the
likelihood on pure noise.
"""
import math

import numpy as np
import pytest

import synth
from tests import bruteforce as bf


def _planes32(oracle_mod, st):
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    return psi.astype(np.float32), phi.astype(np.float32)


def _assert_same(a, b, rel=1e-12):
    np.testing.assert_array_equal(a["vel_idx"], b["vel_idx"])
    np.testing.assert_array_equal(a["n_obs"], b["n_obs"])
    np.testing.assert_array_equal(a["keep"].astype(np.uint64), b["keep"].astype(np.uint64))
    for f in ("lh", "flux", "lh_raw"):
        x, y = a[f], b[f]
        fin = np.isfinite(y)
        np.testing.assert_array_equal(np.isfinite(x), fin)
        np.testing.assert_allclose(x[fin], y[fin], rtol=rel, atol=rel)


@pytest.mark.parametrize("seed,sigmag,k,min_obs", [
    (1, 1, 3, 1), (2, 1, 1, 2), (3, 0, 4, 1), (4, 1, 5, 3), (5, 0, 2, 4)])
def test_search_matches_bruteforce(oracle_mod, seed, sigmag, k, min_obs):
    st = synth.tiny_stack(seed, W=9, H=8, T=5, k=3, n_vel=9, mask_rate=0.2)
    psi, phi = _planes32(oracle_mod, st)
    o = oracle_mod.search(psi, phi, st.times, st.vels, k=k, min_obs=min_obs,
                          sigmag=sigmag)
    b = bf.search(psi, phi, st.times, st.vels, k, min_obs, sigmag=sigmag)
    _assert_same(o, b)


def test_region_and_duplicates(oracle_mod):
    """A start-pixel region, and duplicated velocities: exact ties are
    broken toward the smaller velocity index."""
    st = synth.tiny_stack(12, W=10, H=9, T=4, n_vel=5)
    vels = np.concatenate([st.vels, st.vels[::-1], np.zeros((2, 2), np.float32)])
    psi, phi = _planes32(oracle_mod, st)
    region = (2, 1, 8, 7)
    o = oracle_mod.search(psi, phi, st.times, vels, k=6, min_obs=1,
                          region=region)
    b = bf.search(psi, phi, st.times, vels, 6, 1, region=region)
    _assert_same(o, b)
    assert o["lh"].shape == (6, 6, 6)


def test_closed_form_config1_source(oracle_mod):
    """Noise-free source of flux f injected pixel-centred on the rounded
    track of a grid velocity, variance v: L = f sqrt(T S2 / v), S2 = sum P^2.
    For sigma = 1 on 7x7, f = 100, T = 5, v = 1 this is 63.1189907761; the
    constant lightcurve passes sigma_G untouched, so L' = L."""
    st = synth.make_config(1)
    psf = st.psf
    r = psf.shape[0] // 2
    f, var = 100.0, 1.0
    T, H, W = st.T, st.H, st.W
    vi = 16 * 2 + 12                   # angle 2*2pi/16, speed 16 px/day
    off = oracle_mod.offsets(st.times, st.vels)[vi]
    x0, y0 = 20, 30
    sci = np.zeros((T, H, W), np.float32)
    stamp = (f * psf.astype(np.float64)).astype(np.float32)
    for i in range(T):
        cx, cy = x0 + off[i, 0], y0 + off[i, 1]
        sci[i, cy - r:cy + r + 1, cx - r:cx + r + 1] += stamp
    psi, phi = oracle_mod.planes(sci, np.full((T, H, W), var, np.float32),
                                 None, psf)
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    # 0.079680139932 and 63.1189907761 hold for the FP64 PSF; the stored
    # float32 PSF moves them in the ninth digit.
    assert abs(s2 - 0.079680139932) < 1e-9
    expected = f * math.sqrt(T * s2 / var)
    assert abs(expected - 63.1189907761) < 1e-6
    o = oracle_mod.search(psi.astype(np.float32), phi.astype(np.float32),
                          st.times, st.vels, k=1, min_obs=4, sigmag=1,
                          region=(x0, y0, x0 + 1, y0 + 1))
    assert o["lh"][0, 0, 0] == pytest.approx(expected, rel=2e-7)
    assert o["lh_raw"][0, 0, 0] == pytest.approx(expected, rel=2e-7)
    assert int(o["keep"][0, 0, 0]) == (1 << T) - 1
    win = int(o["vel_idx"][0, 0, 0])
    np.testing.assert_array_equal(oracle_mod.offsets(st.times, st.vels)[win], off)
    assert win <= vi
    # per-epoch SNR nu_i = f sqrt(S2/v) = 28.2276708093
    assert abs(f * math.sqrt(s2 / var) - 28.2276708093) < 1e-6


def test_static_source_translation(oracle_mod):
    """A zero-velocity static source scores the same wherever it sits."""
    psf = synth.gaussian_psf(1.0)
    r = psf.shape[0] // 2
    T, H, W = 5, 40, 40
    times = np.array([0.0, 0.1, 0.2, 1.0, 1.1])
    vels = np.array([[0.0, 0.0], [3.0, 1.0], [-2.0, 2.5]], np.float32)
    res = []
    for (x, y) in [(10, 12), (27, 20), (15, 31)]:
        sci = np.zeros((T, H, W), np.float32)
        sci[:, y - r:y + r + 1, x - r:x + r + 1] = (50.0 * psf).astype(np.float32)
        psi, phi = oracle_mod.planes(sci, np.ones((T, H, W), np.float32), None, psf)
        o = oracle_mod.search(psi.astype(np.float32), phi.astype(np.float32),
                              times, vels, k=3, min_obs=1, sigmag=1,
                              region=(x, y, x + 1, y + 1))
        res.append(o)
    for o in res[1:]:
        _assert_same(o, res[0], rel=0.0)
    assert int(res[0]["vel_idx"][0, 0, 0]) == 0


def test_translation_invariance_all_velocities(oracle_mod):
    """Shifting every plane by d shifts every trajectory result by d
    (outside pixels carry phi = 0 and are invalid in both)."""
    st = synth.tiny_stack(21, W=14, H=12, T=5, n_vel=7, mask_rate=0.1)
    psi, phi = _planes32(oracle_mod, st)
    dy, dx = 3, 5
    T, H, W = psi.shape
    psi2 = np.zeros((T, H + 7, W + 9), np.float32)
    phi2 = np.zeros_like(psi2)
    psi2[:, dy:dy + H, dx:dx + W] = psi
    phi2[:, dy:dy + H, dx:dx + W] = phi
    a = oracle_mod.search(psi, phi, st.times, st.vels, k=4, min_obs=2)
    b = oracle_mod.search(psi2, phi2, st.times, st.vels, k=4, min_obs=2,
                          region=(dx, dy, dx + W, dy + H))
    _assert_same(a, b, rel=0.0)


def test_scale_invariance(oracle_mod):
    """I -> 2I, var -> 4 var leaves L, L' and the keep masks unchanged."""
    st = synth.tiny_stack(22, W=12, H=10, T=6, n_vel=8)
    p1 = _planes32(oracle_mod, st)
    p2 = oracle_mod.planes(st.sci * 2, st.var * 4, st.mask, st.psf)
    p2 = (p2[0].astype(np.float32), p2[1].astype(np.float32))
    a = oracle_mod.search(*p1, st.times, st.vels, k=3, min_obs=2)
    b = oracle_mod.search(*p2, st.times, st.vels, k=3, min_obs=2)
    np.testing.assert_array_equal(a["vel_idx"], b["vel_idx"])
    np.testing.assert_array_equal(a["keep"], b["keep"])
    np.testing.assert_allclose(a["lh"], b["lh"], rtol=1e-13)
    np.testing.assert_allclose(b["flux"], a["flux"] * 2, rtol=1e-13)


def test_epoch_permutation(oracle_mod):
    st = synth.tiny_stack(23, W=12, H=10, T=6, n_vel=8)
    psi, phi = _planes32(oracle_mod, st)
    perm = np.array([3, 0, 5, 1, 4, 2])
    a = oracle_mod.search(psi, phi, st.times, st.vels, k=3, min_obs=2)
    b = oracle_mod.search(psi[perm], phi[perm], st.times[perm], st.vels, k=3,
                          min_obs=2)
    np.testing.assert_array_equal(a["vel_idx"], b["vel_idx"])
    np.testing.assert_allclose(a["lh"], b["lh"], rtol=1e-12)
    ka, kb = a["keep"].astype(np.uint64), b["keep"].astype(np.uint64)
    for j, p in enumerate(perm):
        np.testing.assert_array_equal((ka >> np.uint64(p)) & np.uint64(1),
                                      (kb >> np.uint64(j)) & np.uint64(1))


def test_noise_likelihood_is_unit_normal(oracle_mod):
    """Pure N(0,1) noise with unit variance: for one velocity the plain
    likelihood over start pixels has mean ~0 and variance ~1."""
    rng = np.random.default_rng(31)
    T, H, W = 6, 140, 140
    sci = rng.standard_normal((T, H, W)).astype(np.float32)
    var = np.ones_like(sci)
    psf = synth.gaussian_psf(1.2)
    psi, phi = oracle_mod.planes(sci, var, None, psf)
    times = np.array([0.0, 0.2, 0.4, 1.0, 1.2, 2.0])
    o = oracle_mod.search(psi.astype(np.float32), phi.astype(np.float32),
                          times, np.array([[2.0, 1.5]], np.float32), k=1,
                          min_obs=T, sigmag=0, region=(8, 8, 128, 128))
    L = o["lh"][..., 0].ravel()
    assert abs(L.mean()) < 0.1
    assert abs(L.var() - 1.0) < 0.12


def test_min_obs_and_empty(oracle_mod):
    st = synth.tiny_stack(24, W=10, H=9, T=5, n_vel=6, max_speed=8.0)
    psi, phi = _planes32(oracle_mod, st)
    o = oracle_mod.search(psi, phi, st.times, st.vels, k=6, min_obs=5)
    full = o["vel_idx"] >= 0
    assert np.all(o["n_obs"][full] == 5)
    assert np.all(o["n_obs"][~full] == 0)
    assert np.all(np.isneginf(o["lh"][~full]))
    # an all-masked stack yields only empty slots
    m = np.ones_like(st.mask)
    p2 = oracle_mod.planes(st.sci, st.var, m, st.psf)
    o2 = oracle_mod.search(p2[0].astype(np.float32), p2[1].astype(np.float32),
                           st.times, st.vels, k=2, min_obs=1)
    assert np.all(o2["vel_idx"] == -1) and np.all(np.isneginf(o2["lh"]))
    # an empty region is not an error
    o3 = oracle_mod.search(psi, phi, st.times, st.vels, k=2, region=(3, 3, 3, 5))
    assert o3["lh"].shape == (2, 0, 2)


def test_offsets_round_half_up(oracle_mod):
    times = np.array([5.0, 5.25, 6.0])          # measured from the earliest
    vels = np.array([[10.0, -10.0], [0.5, -0.5], [0.3, -0.3]], np.float32)
    off = oracle_mod.offsets(times, vels)
    assert off[0].tolist() == [[0, 0], [3, -2], [10, -10]]
    assert off[1].tolist() == [[0, 0], [0, 0], [1, 0]]
    assert off[2].tolist() == [[0, 0], [0, 0], [0, 0]]
