"""Seeded generator: determinism and the workload shapes it promises."""
import hashlib

import numpy as np

import synth


def _digest(st):
    h = hashlib.sha256()
    for a in (st.sci, st.var, st.mask, st.psf, st.times, st.vels):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_same_seed_same_arrays():
    a = synth.make_config(2, size=(96, 80), n_vel=(8, 8))
    b = synth.make_config(2, size=(96, 80), n_vel=(8, 8))
    assert _digest(a) == _digest(b)
    c = synth.make_config(2, seed=77, size=(96, 80), n_vel=(8, 8))
    assert _digest(a) != _digest(c)


def test_config_shapes():
    c1 = synth.make_config(1)
    assert c1.sci.shape == (5, 64, 64) and c1.psf.shape == (7, 7)
    assert c1.vels.shape == (256, 2) and c1.mask is None
    assert np.all(c1.var == 1.0) and c1.times[0] == 0.0 and c1.times.max() <= 1.0
    t = synth.night_times(26, 3)
    nights = np.floor(t + 0.5).astype(int)
    assert [int(np.sum(nights == n)) for n in range(3)] == [9, 9, 8]
    assert np.allclose(np.diff(t[:9]), 5 / 1440)
    assert synth.psf_size(1.0) == 7 and synth.psf_size(1.4) == 9 and synth.psf_size(1.6) == 11
    p = synth.gaussian_psf(1.4)
    assert abs(float(p.astype(np.float64).sum()) - 1.0) < 1e-6
    assert np.array_equal(p, p.T) and np.array_equal(p, p[::-1])


def test_sources_stay_inside():
    st = synth.make_config(2, size=(1200, 700), n_vel=(4, 4))
    r = st.psf.shape[0] // 2
    for s in st.sources:
        for t in st.times:
            x, y = s["x0"] + s["vx"] * t, s["y0"] + s["vy"] * t
            assert r + 1 <= x <= st.W - 2 - r and r + 1 <= y <= st.H - 2 - r
    assert 0.005 < st.mask.mean() < 0.015
