"""Pins for the oracle's likelihood planes (Section 3: psi/phi images).

Each check ties the oracle to something other than itself: a library
correlation routine, the delta-PSF special case, masking invariances and the
closed form of a noise-free pixel-centred source.
"""
import numpy as np
import pytest

import synth
from tests import bruteforce as bf


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_planes_match_library_correlation(oracle_mod, seed):
    st = synth.tiny_stack(seed, W=13, H=11, T=3, k=5, mask_rate=0.2)
    rng = np.random.default_rng(seed)
    psf = rng.uniform(0.0, 1.0, size=(5, 5)).astype(np.float32)  # asymmetric
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, psf)
    rpsi, rphi = bf.planes(st.sci, st.var, st.mask, psf)
    np.testing.assert_allclose(psi, rpsi, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(phi, rphi, rtol=1e-12, atol=1e-12)


def test_correlation_orientation():
    """A PSF with a single tap at row r+1 (b = +1) reads the pixel below:
    psi(y, x) = P * I(y+1, x) * w(y+1, x).  Pins correlation vs convolution."""
    import oracle
    T, H, W = 1, 6, 7
    rng = np.random.default_rng(0)
    sci = rng.normal(size=(T, H, W)).astype(np.float32)
    var = rng.uniform(1, 2, size=(T, H, W)).astype(np.float32)
    psf = np.zeros((3, 3), np.float32)
    psf[2, 1] = 0.5
    psi, phi = oracle.planes(sci, var, None, psf)
    exp = np.zeros((H, W))
    exp[:-1] = 0.5 * sci[0, 1:].astype(np.float64) / var[0, 1:].astype(np.float64)
    np.testing.assert_allclose(psi[0], exp, rtol=1e-15, atol=0)
    expf = np.zeros((H, W))
    expf[:-1] = 0.25 / var[0, 1:].astype(np.float64)
    np.testing.assert_allclose(phi[0], expf, rtol=1e-15, atol=0)


def test_delta_psf_gives_inverse_variance(oracle_mod):
    st = synth.tiny_stack(5, mask_rate=0.3)
    psf = np.zeros((3, 3), np.float32)
    psf[1, 1] = 1.0
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, psf)
    ok = st.mask == 0
    np.testing.assert_array_equal(psi[~ok], 0.0)
    np.testing.assert_array_equal(phi[~ok], 0.0)
    np.testing.assert_allclose(psi[ok], st.sci[ok] / st.var[ok].astype(np.float64), rtol=1e-15)
    np.testing.assert_allclose(phi[ok], 1.0 / st.var[ok].astype(np.float64), rtol=1e-15)


@pytest.mark.parametrize("fill", [np.nan, 1e30, -np.inf])
def test_masked_values_never_enter(oracle_mod, fill):
    a = synth.tiny_stack(7, mask_rate=0.25)
    b = synth.tiny_stack(7, mask_rate=0.25, masked_fill=fill)
    pa = oracle_mod.planes(a.sci, a.var, a.mask, a.psf)
    pb = oracle_mod.planes(b.sci, b.var, b.mask, b.psf)
    np.testing.assert_array_equal(pa[0], pb[0])
    np.testing.assert_array_equal(pa[1], pb[1])


def test_mask_equals_zero_weight(oracle_mod):
    """Masking a pixel is the same as giving it no usable variance."""
    st = synth.tiny_stack(8, mask_rate=0.25)
    var2 = st.var.copy()
    var2[st.mask != 0] = 0.0
    pa = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    pb = oracle_mod.planes(st.sci, var2, None, st.psf)
    np.testing.assert_array_equal(pa[0], pb[0])
    np.testing.assert_array_equal(pa[1], pb[1])


def test_scaling(oracle_mod):
    """I -> cI, var -> c^2 var gives psi -> psi/c, phi -> phi/c^2 (c a power
    of two, so the scaled float32 inputs are exact)."""
    st = synth.tiny_stack(9)
    c = 2.0
    p1 = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    p2 = oracle_mod.planes((st.sci.astype(np.float64) * c).astype(np.float32),
                           (st.var.astype(np.float64) * c * c).astype(np.float32),
                           st.mask, st.psf)
    np.testing.assert_allclose(p2[0] * c, p1[0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(p2[1] * c * c, p1[1], rtol=1e-13, atol=1e-13)


def test_closed_form_pixel_centred_source(oracle_mod):
    """Noise-free source f*P centred on a pixel, constant variance v:
    psi = f*S2/v and phi = S2/v there, S2 = sum P^2."""
    psf = synth.gaussian_psf(1.4)
    k = psf.shape[0]
    r = k // 2
    f, v = 250.0, 4.0
    H = W = 40
    sci = np.zeros((1, H, W), np.float32)
    sci[0, 20 - r:20 + r + 1, 17 - r:17 + r + 1] = (f * psf.astype(np.float64)).astype(np.float32)
    var = np.full((1, H, W), v, np.float32)
    psi, phi = oracle_mod.planes(sci, var, None, psf)
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    fP = (f * psf.astype(np.float64)).astype(np.float32).astype(np.float64)
    assert abs(psi[0, 20, 17] - np.sum(psf * fP) / v) < 1e-12
    assert abs(psi[0, 20, 17] - f * s2 / v) < 1e-5 * f * s2 / v
    assert abs(phi[0, 20, 17] - s2 / v) < 1e-15
    # phi is the same everywhere the whole footprint is inside the image
    np.testing.assert_allclose(phi[0, r:H - r, r:W - r], s2 / v, rtol=1e-14)
    # edges lose the out-of-image taps
    assert phi[0, 0, 0] < s2 / v
