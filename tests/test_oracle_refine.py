"""Pins for the oracle's bilinear refinement objective and its gradient.

Central finite differences of the FP64 objective, a library bilinear
sampler, the reduction to the grid search at integer positions, and the
(linear) dependence on the psi planes.
"""
import numpy as np
import pytest

import synth
from tests import bruteforce as bf

H2 = 2.0 ** -13   # exactly representable step for float32 parameters


def _smooth_planes(seed, T=6, H=24, W=28):
    rng = np.random.default_rng(seed)
    psi = rng.normal(size=(T, H, W)).astype(np.float32) + 2.0
    phi = rng.uniform(0.5, 1.5, size=(T, H, W)).astype(np.float32)
    return psi, phi


def _far_from_integers(params, times, margin):
    t = times - times.min()
    x = params[:, 0:1] + params[:, 2:3] * t[None, :]
    y = params[:, 1:2] + params[:, 3:4] * t[None, :]
    dx = np.abs(x - np.round(x))
    dy = np.abs(y - np.round(y))
    m = margin * np.maximum(1.0, t)[None, :]
    return np.all(dx > m, axis=1) & np.all(dy > m, axis=1)


def test_gradient_matches_central_differences(oracle_mod):
    psi, phi = _smooth_planes(1)
    times = np.array([0.0, 0.13, 0.31, 1.07, 1.29, 2.02])
    rng = np.random.default_rng(2)
    n = 400
    params = np.stack([rng.uniform(4, 20, n), rng.uniform(4, 16, n),
                       rng.uniform(-2.5, 2.5, n), rng.uniform(-2.5, 2.5, n)],
                      axis=1).astype(np.float32)
    params = params[_far_from_integers(params.astype(np.float64), times, 4 * H2)]
    assert len(params) > 20
    keep = rng.integers(1, 2 ** 6, size=len(params)).astype(np.uint64)
    lh, gp = oracle_mod.refine(psi, phi, times, params, keep,
                               grad_lh=np.ones(len(params)))
    for j in range(4):
        pp, pm = params.copy(), params.copy()
        pp[:, j] += np.float32(H2)
        pm[:, j] -= np.float32(H2)
        step = pp[:, j].astype(np.float64) - pm[:, j].astype(np.float64)
        fd = (oracle_mod.refine(psi, phi, times, pp, keep)
              - oracle_mod.refine(psi, phi, times, pm, keep)) / step
        scale = np.maximum(np.abs(gp[:, j]), 1e-3)
        assert np.max(np.abs(fd - gp[:, j]) / scale) < 1e-6, j


def test_upstream_gradient_scales(oracle_mod):
    psi, phi = _smooth_planes(3)
    times = np.linspace(0, 2, 6)
    params = np.array([[10.3, 8.6, 1.1, -0.7], [5.2, 12.4, -2.1, 0.4]], np.float32)
    _, g1 = oracle_mod.refine(psi, phi, times, params, grad_lh=np.ones(2))
    _, g2 = oracle_mod.refine(psi, phi, times, params, grad_lh=np.array([2.5, -1.0]))
    np.testing.assert_allclose(g2, g1 * np.array([[2.5], [-1.0]]), rtol=1e-15)


def test_bilinear_matches_library(oracle_mod):
    """T = 1: L = B(psi)/sqrt(B(phi)) with B the library bilinear sampler
    (zero outside the image), including points hanging over the edges."""
    rng = np.random.default_rng(4)
    psi = rng.normal(size=(1, 9, 11)).astype(np.float32)
    phi = rng.uniform(0.5, 2.0, size=(1, 9, 11)).astype(np.float32)
    pts = np.concatenate([rng.uniform(0, 9.5, (40, 1)), rng.uniform(0, 7.5, (40, 1)),
                          np.zeros((40, 2))], axis=1)
    pts = np.concatenate([pts, [[-0.4, 3.2, 0, 0], [10.3, 8.6, 0, 0],
                                [4.0, 5.0, 0, 0], [0.0, 0.0, 0, 0]]]).astype(np.float32)
    lh = oracle_mod.refine(psi, phi, np.zeros(1), pts)
    for c, p in enumerate(pts):
        x, y = float(p[0]), float(p[1])
        ref = bf.bilinear(psi[0], x, y) / np.sqrt(bf.bilinear(phi[0], x, y))
        assert lh[c] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_integer_positions_reduce_to_grid_search(oracle_mod):
    """At integer start pixels and velocities whose tracks land on pixel
    centres the objective is the plain trajectory likelihood."""
    st = synth.tiny_stack(41, W=16, H=14, T=4, mask_rate=0.0)
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    psi, phi = psi.astype(np.float32), phi.astype(np.float32)
    times = np.array([0.0, 1.0, 2.0, 3.0])
    vels = np.array([[1.0, 2.0], [-2.0, 1.0], [3.0, -1.0], [0.0, 0.0]], np.float32)
    for v in range(len(vels)):
        for (x, y) in [(3, 2), (8, 5), (12, 10), (6, 7)]:
            s = oracle_mod.search(psi, phi, times, vels[v:v + 1], k=1, min_obs=1,
                                  sigmag=0, region=(x, y, x + 1, y + 1))
            lh = oracle_mod.refine(psi, phi, times,
                                   np.array([[x, y, vels[v, 0], vels[v, 1]]], np.float32))
            if s["vel_idx"][0, 0, 0] < 0:
                continue
            assert lh[0] == pytest.approx(s["lh_raw"][0, 0, 0], rel=1e-13)


def test_plane_gradients(oracle_mod):
    """L is linear in psi (exact check) and smooth in phi (central FD)."""
    psi, phi = _smooth_planes(5, T=3, H=12, W=12)
    times = np.array([0.0, 0.5, 1.0])
    params = np.array([[4.3, 5.6, 1.7, 0.9]], np.float32)
    lh, _, gpsi, gphi = oracle_mod.refine(psi, phi, times, params,
                                          grad_lh=np.ones(1), want_planes=True)
    nz = np.argwhere(gpsi != 0)
    assert len(nz) == 12            # 4 taps x 3 epochs
    for (t, y, x) in nz[:6]:
        d = np.float32(0.25)
        p2 = psi.copy()
        p2[t, y, x] += d
        l2 = oracle_mod.refine(p2, phi, times, params)
        assert (l2[0] - lh[0]) / float(d) == pytest.approx(gpsi[t, y, x], rel=1e-9)
        h = np.float32(2.0 ** -12)
        fp, fm = phi.copy(), phi.copy()
        fp[t, y, x] += h
        fm[t, y, x] -= h
        fd = (oracle_mod.refine(psi, fp, times, params)[0]
              - oracle_mod.refine(psi, fm, times, params)[0]) / (2 * float(h))
        assert fd == pytest.approx(gphi[t, y, x], rel=1e-6)


def test_off_image_candidate(oracle_mod):
    psi, phi = _smooth_planes(6)
    params = np.array([[-50.0, -50.0, 0.0, 0.0]], np.float32)
    lh, gp = oracle_mod.refine(psi, phi, np.linspace(0, 1, 6), params,
                               grad_lh=np.ones(1))
    assert lh[0] == 0.0 and np.all(gp == 0.0)
