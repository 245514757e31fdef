"""Pins for the oracle's targeted evaluation (explicit trajectories with
real-valued starts): pure-Python brute force, and reduction to the
exhaustive search at integer starts."""
import math

import numpy as np
import pytest

import synth
from tests import bruteforce as BF

SG = dict(q_lo=0.25, q_hi=0.75, coeff=0.7413, n_sigma=2.0)


def _planes(oracle_mod, st):
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    return psi.astype(np.float32), phi.astype(np.float32)


@pytest.mark.parametrize("seed,T,sigmag,min_obs", [(41, 5, 1, 1), (42, 9, 1, 4),
                                                   (43, 13, 0, 3), (44, 26, 1, 20)])
def test_score_bruteforce(oracle_mod, seed, T, sigmag, min_obs):
    st = synth.tiny_stack(seed, W=17, H=13, T=T, mask_rate=0.2, masked_fill=np.nan)
    psi, phi = _planes(oracle_mod, st)
    rng = np.random.default_rng(seed)
    n = 150
    prm = np.stack([rng.uniform(-3, 19, n), rng.uniform(-3, 15, n),
                    rng.uniform(-8, 8, n), rng.uniform(-8, 8, n)], 1).astype(np.float32)
    prm[:10, :2] = np.round(prm[:10, :2]) + 0.5      # half-pixel starts
    got = oracle_mod.score(psi, phi, st.times, prm, min_obs=min_obs, sigmag=sigmag, **SG)
    for j in range(n):
        r = BF.trajectory_real(psi, phi, st.times, prm[j], sigmag, **SG)
        if r is None or r["n_obs"] < min_obs or not math.isfinite(r["lh"]):
            assert np.isneginf(got["lh"][j]) and got["keep"][j] == 0, j
            assert got["n_obs"][j] == (0 if r is None else r["n_obs"])
            continue
        assert got["n_obs"][j] == r["n_obs"]
        assert int(got["keep"][j]) == r["keep"], j
        assert got["lh"][j] == pytest.approx(r["lh"], rel=1e-12, abs=1e-12)
        assert got["flux"][j] == pytest.approx(r["flux"], rel=1e-12, abs=1e-12)
        assert got["lh_raw"][j] == pytest.approx(r["lh_raw"], rel=1e-12, abs=1e-12)


def test_score_reduces_to_search_at_integer_starts(oracle_mod):
    st = synth.tiny_stack(45, W=21, H=11, T=11, n_vel=9, mask_rate=0.1)
    psi, phi = _planes(oracle_mod, st)
    p = dict(k=1, min_obs=5, sigmag=1, **SG)
    pts, rows = [], []
    for v in range(len(st.vels)):
        for y in range(0, st.H, 2):
            for x in range(0, st.W, 3):
                pts.append((x, y, v))
                rows.append([x, y, st.vels[v, 0], st.vels[v, 1]])
    got = oracle_mod.score(psi, phi, st.times, np.array(rows, np.float32), **p)
    for j, (x, y, v) in enumerate(pts):
        r = oracle_mod.search(psi, phi, st.times, st.vels[v:v + 1],
                              region=(x, y, x + 1, y + 1), **p)
        assert got["lh"][j] == r["lh"][0, 0, 0] or (
            np.isneginf(got["lh"][j]) and np.isneginf(r["lh"][0, 0, 0])), (x, y, v)
        if np.isfinite(r["lh"][0, 0, 0]):
            assert int(got["keep"][j]) == int(r["keep"][0, 0, 0])
            assert got["n_obs"][j] == r["n_obs"][0, 0, 0]
            assert got["flux"][j] == r["flux"][0, 0, 0]
            assert got["lh_raw"][j] == r["lh_raw"][0, 0, 0]


def test_score_closed_form_source(oracle_mod):
    """Noise-free pixel-centred source: the targeted L at its true track is
    f sqrt(T S2 / v) (the tiny configuration's closed form)."""
    st = synth.make_config(1)
    # zero the noise: rebuild the stack with the same source and no noise
    s = st.sources[0]
    T, H, W = st.sci.shape
    sci = np.zeros_like(st.sci)
    for i, t in enumerate(st.times):
        x = int(math.floor(s["x0"] + s["vx"] * t + 0.5))
        y = int(math.floor(s["y0"] + s["vy"] * t + 0.5))
        r = st.psf.shape[0] // 2
        sci[i, y - r:y + r + 1, x - r:x + r + 1] += s["flux"] * st.psf
    psi, phi = oracle_mod.planes(sci, st.var, None, st.psf)
    got = oracle_mod.score(psi.astype(np.float32), phi.astype(np.float32), st.times,
                           np.array([[s["x0"], s["y0"], s["vx"], s["vy"]]], np.float32),
                           min_obs=1, sigmag=1, **SG)
    s2 = float(np.sum(st.psf.astype(np.float64) ** 2))
    assert got["lh"][0] == pytest.approx(s["flux"] * math.sqrt(T * s2), rel=1e-6)
    assert int(got["keep"][0]) == (1 << T) - 1
