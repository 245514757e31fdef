"""GPU: median coadded stamps and the central-moment cut (Section 3.3)
against the oracle.  Coadds are selections and one binary32 halving, so they
compare exactly; moments are FP64 sums in a different order (relative
1e-12); pass flags agree except where the oracle's moment lies within 1e-9
of a limit."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03296_amd as kbm
    kbm.lib()
    return kbm


def _cu(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(oracle_mod, got, sci, var, mask, times, prm, radius, keep=None):
    ref = oracle_mod.stamps(sci, var, mask, times, prm, radius=radius, keep=keep)
    co = got["coadd"].cpu().numpy()
    assert np.array_equal(co, ref)
    m_ref = oracle_mod.stamp_moments(ref)
    m = got["moments"].cpu().numpy()
    fin = np.isfinite(m_ref)
    assert np.array_equal(np.isfinite(m), fin)
    assert np.all(np.abs(m[fin] - m_ref[fin]) <= 1e-12 * np.maximum(np.abs(m_ref[fin]), 1.0))
    p_ref = oracle_mod.stamp_pass(m_ref)
    p = got["passed"].cpu().numpy()
    lim = np.array(oracle_mod.STAMP_LIMITS)
    vals = np.abs(m_ref[:, 1:])
    near = np.any(np.abs(vals - lim[None, :]) <= 1e-9 * lim[None, :], axis=1)
    assert np.all((p == p_ref) | near)
    return ref, m_ref, p_ref


@pytest.mark.parametrize("seed,T,radius,use_keep", [(71, 5, 2, False), (72, 13, 10, True),
                                                    (73, 26, 10, False), (74, 40, 6, True),
                                                    (75, 60, 15, False)])
def test_stamps_match_oracle(kbm, oracle_mod, seed, T, radius, use_keep):
    st = synth.tiny_stack(seed, W=57, H=43, T=T, mask_rate=0.15, masked_fill=np.nan)
    st.var[0, :5, :5] = 0.0
    rng = np.random.default_rng(seed)
    n = 200
    prm = np.stack([rng.uniform(-12, 69, n), rng.uniform(-12, 55, n),
                    rng.uniform(-9, 9, n), rng.uniform(-9, 9, n)], 1).astype(np.float32)
    prm[:20, 2:] = 0.0                        # static
    keep = rng.integers(0, 2 ** min(T, 62), n).astype(np.int64) if use_keep else None
    got = kbm.stamps(_cu(st.sci), _cu(st.var), _cu(st.mask), st.times, _cu(prm),
                     keep=_cu(keep), radius=radius)
    _compare(oracle_mod, got, st.sci, st.var, st.mask, st.times, prm, radius,
             None if keep is None else keep.astype(np.uint64))


def test_stamps_of_search_candidates(kbm, oracle_mod):
    """Search a crop of the CCD stack, take the top slots and coadd their
    stamps with the search's keep masks: the oracle agrees."""
    st = synth.make_config(2, size=(400, 300), n_vel=(16, 16))
    p = st.params
    sci, var, mask = _cu(st.sci), _cu(st.var), _cu(st.mask)
    psi, phi = kbm.make_planes(sci, var, mask, st.psf, st.times)
    sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=True)
    res = kbm.search(psi, phi, st.times, st.vels, sp)
    cand = kbm.extract_top(res, st.vels, 500)
    got = kbm.stamps(sci, var, mask, st.times, cand["params"].contiguous(),
                     keep=cand["keep"].contiguous(), radius=10)
    _compare(oracle_mod, got, st.sci, st.var, st.mask, st.times,
             cand["params"].cpu().numpy(), 10, cand["keep"].cpu().numpy().view(np.uint64))


def test_stamps_noise_free_source(kbm, oracle_mod):
    """A noise-free source drawn with the PSF at the trajectory's pixel in
    every epoch: the coadd is flux x PSF, the odd moments vanish, xx = yy is
    the PSF's own second moment, and the stamp passes the cut."""
    st = synth.make_config(1)
    s0 = st.sources[0]
    T, H, W = st.sci.shape
    r = st.psf.shape[0] // 2
    sci = np.zeros_like(st.sci)
    for i, t in enumerate(st.times):
        x = int(np.floor(s0["x0"] + s0["vx"] * t + 0.5))
        y = int(np.floor(s0["y0"] + s0["vy"] * t + 0.5))
        sci[i, y - r:y + r + 1, x - r:x + r + 1] += np.float32(s0["flux"]) * st.psf
    truth = np.array([[s0["x0"], s0["y0"], s0["vx"], s0["vy"]]], np.float32)
    got = kbm.stamps(_cu(sci), _cu(st.var), None, st.times, _cu(truth), radius=10)
    co, m_ref, _ = _compare(oracle_mod, got, sci, st.var, None, st.times, truth, 10)
    want = np.zeros((21, 21), np.float32)
    want[10 - r:11 + r, 10 - r:11 + r] = np.float32(s0["flux"]) * st.psf
    assert np.array_equal(co[0], want)
    m = got["moments"].cpu().numpy()[0]
    p = want.astype(np.float64)          # the float32 values the coadd holds
    d = np.arange(-10, 11, dtype=np.float64)
    xx = float((p * d[None, :] ** 2).sum() / p.sum())
    assert abs(m[1]) < 1e-12 and abs(m[2]) < 1e-12 and abs(m[3]) < 1e-12
    assert m[4] == pytest.approx(xx, rel=1e-9) and m[5] == pytest.approx(xx, rel=1e-9)
    assert bool(got["passed"][0])


def test_moment_limits_strict_on_gpu(kbm, oracle_mod):
    """Coadds whose moments sit exactly on a limit (x = 0.5, xy = 1.5,
    xx = yy = 36.5; every sum exact in binary64 in any order) fail the cut
    on the GPU as in the oracle, and their twins nudged inside pass.  Three
    identical epochs and a static trajectory make the median coadd the
    pattern itself."""
    from tests.test_oracle_stamps import _limit_stamps
    pats = []
    for _, s in _limit_stamps():
        pats.append(s)
        s2 = s.copy()
        s2[10, 10] += 1e-3
        pats.append(s2)
    T, r = 3, 10
    W = 21 * len(pats) + 10
    H = 31
    img = np.zeros((H, W), np.float32)
    prm = []
    for j, s in enumerate(pats):
        x0 = 5 + 21 * j
        img[5:26, x0:x0 + 21] = s.astype(np.float32)
        prm.append([x0 + 10, 15, 0.0, 0.0])
    sci = np.ascontiguousarray(np.broadcast_to(img, (T, H, W)))
    var = np.ones((T, H, W), np.float32)
    times = np.array([0.0, 0.01, 0.02])
    prm = np.array(prm, np.float32)
    got = kbm.stamps(_cu(sci), _cu(var), None, times, _cu(prm), radius=r)
    ref, m_ref, p_ref = _compare(oracle_mod, got, sci, var, None, times, prm, r)
    assert list(p_ref) == [False, True] * (len(pats) // 2)
    assert np.array_equal(got["passed"].cpu().numpy(), p_ref)
