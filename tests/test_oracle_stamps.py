"""Pins for the oracle's median coadded stamps and central moments
(Section 3.3): pure-Python medians, closed forms, robustness of the median
to artifacts in a minority of epochs, keep masks and image edges."""
import math

import numpy as np
import pytest

import synth

F32 = np.float32


def _bf_stamp(sci, var, mask, times, prm, r, keep=None):
    T, H, W = sci.shape
    t0 = min(times)
    k = 2 * r + 1
    out = np.zeros((k, k), np.float32)
    x0, y0, vx, vy = (float(F32(v)) for v in prm)
    for a in range(k):
        for b in range(k):
            vals = []
            for i in range(T):
                if keep is not None and not (keep >> i) & 1:
                    continue
                cx = math.floor(x0 + vx * (float(times[i]) - float(t0)) + 0.5)
                cy = math.floor(y0 + vy * (float(times[i]) - float(t0)) + 0.5)
                y, x = cy + a - r, cx + b - r
                if not (0 <= x < W and 0 <= y < H):
                    continue
                if mask is not None and mask[i, y, x]:
                    continue
                s, v = sci[i, y, x], var[i, y, x]
                if not (np.isfinite(s) and np.isfinite(v) and v > 0):
                    continue
                vals.append(F32(s))
            if not vals:
                continue
            vals.sort()
            n = len(vals)
            out[a, b] = vals[n // 2] if n % 2 else F32(F32(vals[n // 2 - 1] + vals[n // 2]) / F32(2))
    return out


@pytest.mark.parametrize("seed,T,r", [(61, 5, 2), (62, 8, 3), (63, 11, 4)])
def test_stamps_bruteforce(oracle_mod, seed, T, r):
    st = synth.tiny_stack(seed, W=19, H=15, T=T, mask_rate=0.25, masked_fill=np.nan)
    st.var[0, 3, 4] = -1.0
    rng = np.random.default_rng(seed)
    prm = np.stack([rng.uniform(-3, 21, 12), rng.uniform(-3, 17, 12),
                    rng.uniform(-6, 6, 12), rng.uniform(-6, 6, 12)], 1).astype(np.float32)
    keep = rng.integers(0, 2 ** T, 12).astype(np.uint64)
    got = oracle_mod.stamps(st.sci, st.var, st.mask, st.times, prm, radius=r)
    gotk = oracle_mod.stamps(st.sci, st.var, st.mask, st.times, prm, radius=r, keep=keep)
    for j in range(12):
        assert np.array_equal(got[j], _bf_stamp(st.sci, st.var, st.mask, st.times, prm[j], r))
        assert np.array_equal(gotk[j], _bf_stamp(st.sci, st.var, st.mask, st.times, prm[j], r,
                                                 int(keep[j])))


def _gauss_1d(sigma, r):
    d = range(-r, r + 1)
    g = [math.exp(-dd * dd / (2 * sigma * sigma)) for dd in d]
    return list(d), g


@pytest.mark.parametrize("sigma", [0.8, 1.4, 2.5])
def test_moments_of_a_gaussian(oracle_mod, sigma):
    r = 10
    d, g = _gauss_1d(sigma, r)
    stamp = np.outer(g, g)
    m = oracle_mod.stamp_moments(stamp)
    xx = math.fsum(dd * dd * gg for dd, gg in zip(d, g)) / math.fsum(g)
    assert m[0] == pytest.approx(math.fsum(g) ** 2, rel=1e-14)
    assert abs(m[1]) < 1e-14 and abs(m[2]) < 1e-14 and abs(m[3]) < 1e-14
    assert m[4] == pytest.approx(xx, rel=1e-13) and m[5] == pytest.approx(xx, rel=1e-13)
    assert bool(oracle_mod.stamp_pass(m))
    # moved by one pixel in x: the x moment is exactly the shift
    shifted = np.roll(np.pad(stamp, 1), 1, axis=1)[1:-1, 1:-1]
    ms = oracle_mod.stamp_moments(shifted)
    assert ms[1] == pytest.approx(1.0, abs=1e-3 if sigma > 2 else 1e-9)
    assert not bool(oracle_mod.stamp_pass(ms))


def test_moments_uniform_and_negative(oracle_mod):
    k = 21
    m = oracle_mod.stamp_moments(np.ones((k, k)))
    assert m[4] == pytest.approx((k * k - 1) / 12.0, rel=1e-14)   # 36.67 > 36.5
    assert not bool(oracle_mod.stamp_pass(m))
    neg = -np.ones((k, k))
    assert not bool(oracle_mod.stamp_pass(oracle_mod.stamp_moments(neg)))
    assert not bool(oracle_mod.stamp_pass(oracle_mod.stamp_moments(np.zeros((k, k)))))


def test_median_rejects_minority_artifacts(oracle_mod):
    """A static source in 7 epochs with a saturated artifact in 3 of them at
    another place: the median coadd equals the artifact-free one."""
    T, H, W, r = 7, 40, 40, 10
    d, g = _gauss_1d(1.4, 4)
    src = np.outer(g, g).astype(np.float32) * 50
    sci = np.zeros((T, H, W), np.float32)
    sci[:, 16:25, 16:25] += src
    clean = sci.copy()
    sci[:3, 10:13, 26:29] += 1e4
    var = np.ones_like(sci)
    prm = np.array([[20, 20, 0, 0]], np.float32)
    times = np.linspace(0, 1, T)
    a = oracle_mod.stamps(sci, var, None, times, prm, radius=r)
    b = oracle_mod.stamps(clean, var, None, times, prm, radius=r)
    assert np.array_equal(a, b)
    m = oracle_mod.stamp_moments(a[0])
    assert bool(oracle_mod.stamp_pass(m))


def test_stamp_outside_image_is_zero(oracle_mod):
    sci = np.ones((3, 10, 10), np.float32)
    var = np.ones_like(sci)
    prm = np.array([[-50, -50, 0, 0], [4.4, 4.6, 0, 0]], np.float32)
    s = oracle_mod.stamps(sci, var, None, [0, 1, 2], prm, radius=3)
    assert np.all(s[0] == 0)
    assert s[1][3, 3] == 1 and s[1].sum() == 49.0


def _limit_stamps(r=10):
    """Coadds whose moments sit exactly on a limit of the cut (every value
    and sum below is exact in binary64):
      * x = 0.5: equal mass at dx = 0 and dx = +1 on the centre row;
      * xx = 36.5: mass 63.5 at dx = -6 and +6 and 0.5 at dx = -10 and +10
        (total 128): (127 * 36 + 100) / 128 = 36.5;
      * yy = 36.5: the transpose of the previous one;
      * xy = 1.5: mass 7.5 at (dx, dy) = (1, 1) and (-1, -1) and 0.5 at
        (3, 3) and (-3, -3) (total 16): (15 * 1 + 1 * 9) / 16 = 1.5, with
        x = y = 0 and xx = yy = 1.5."""
    k = 2 * r + 1
    out = []
    a = np.zeros((k, k))
    a[r, r] = a[r, r + 1] = 1.0
    out.append(("x", a))
    b = np.zeros((k, k))
    b[r, r - 6] = b[r, r + 6] = 63.5
    b[r, r - 10] = b[r, r + 10] = 0.5
    out.append(("xx", b))
    by = b.T.copy()
    out.append(("yy", by))
    c = np.zeros((k, k))
    c[r + 1, r + 1] = c[r - 1, r - 1] = 7.5
    c[r + 3, r + 3] = c[r - 3, r - 3] = 0.5
    out.append(("xy", c))
    return out


def test_moment_limits_are_strict(oracle_mod):
    """Section 3.3 asks for moments strictly below their limits: a coadd
    whose x moment is exactly 0.5, or whose xx or yy is exactly 36.5, fails
    the cut, as does one whose xy is exactly 1.5, and the same coadd nudged
    just inside passes."""
    for name, s in _limit_stamps():
        m = oracle_mod.stamp_moments(s)
        col = {"x": 1, "xy": 3, "xx": 4, "yy": 5}[name]
        lim = {"x": 0.5, "xy": 1.5, "xx": 36.5, "yy": 36.5}[name]
        assert m[col] == lim, (name, m)
        assert not bool(oracle_mod.stamp_pass(m)), name
        # nudge: a little more mass at the centre pulls the moment inside
        s2 = s.copy()
        s2[10, 10] += 1e-6
        m2 = oracle_mod.stamp_moments(s2)
        assert m2[col] < lim
        assert bool(oracle_mod.stamp_pass(m2)), (name, m2)
    # |x| with a negative moment exactly at the limit fails as well
    s = np.zeros((21, 21))
    s[10, 10] = s[10, 9] = 1.0
    m = oracle_mod.stamp_moments(s)
    assert m[1] == -0.5 and not bool(oracle_mod.stamp_pass(m))
