"""Parity at full size, in the launch configuration bench.py times.

* The DECam-CCD stack (2048 x 4096, T = 26 over 3 nights, 128 x 128
  velocities, K = 8, sigma_G on, min_obs 20) searched by the batched
  persistent kernel with its default schedule.  Both sides read the oracle's
  planes rounded to float32 (protocol B).  Sampled start pixels (every
  injected source's start, random pixels, image corners and edges) are
  re-searched by the oracle one pixel at a time; properties that hold at
  every pixel are checked on the whole result.
* The full-pipeline stack (4096 x 4096, T = 60 over 5 nights, 64 x 64
  velocities): its packed planes (8 GB) exceed one 32-bit buffer
  descriptor, so the search reads them through two; sampled pixels against
  the oracle.
* The batched recipe (62 stacks, sides drawn independently, T in [10, 30],
  PSF sigma in [1, 2], 64 x 64 velocities, K = 8) at reduced image sides:
  the persistent kernel against the per-stack search (bit-identical) and,
  on sampled pixels of every stack, against the oracle.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests import parity as P

pytestmark = pytest.mark.gpu

PKEYS = ("min_obs", "sigmag", "q_lo", "q_hi", "coeff", "n_sigma")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_03296_amd as kbm
    kbm.lib()
    return kbm


def _np(res):
    return P.to_np(res)


def _pixel_check(oracle_mod, psi, phi, st, p, g, pixels, fp64=None):
    """Oracle search of each sampled pixel vs the GPU slots there; with
    ``fp64`` (a dict) given, also certify every GPU slot's binary32 keep
    decisions against the FP64 decision and accumulate the counts."""
    n_ties = 0
    for (x, y) in pixels:
        ref = oracle_mod.search(psi, phi, st.times, st.vels,
                                region=(x, y, x + 1, y + 1), **p)
        sub = {k: v[y:y + 1, x:x + 1] for k, v in g.items()}

        def single(yy, xx, v, x=x, y=y):
            o = oracle_mod.search(psi, phi, st.times, st.vels[v:v + 1], k=1,
                                  region=(x, y, x + 1, y + 1),
                                  **{k: p[k] for k in PKEYS})
            return float(o["lh"][0, 0, 0])
        stats = P.compare_search(sub, ref, single, max_tie_frac=1.0)
        n_ties += stats["tie_swaps"]
        if fp64 is not None and p["sigmag"]:
            c = P.certify_fp64(oracle_mod, sub, psi, phi, st.times, st.vels, p, (x, y))
            for k in ("slots", "bits_differ", "slots_differ"):
                fp64[k] = fp64.get(k, 0) + c[k]
            fp64["worst_ratio"] = max(fp64.get("worst_ratio", 0.0), c["worst_ratio"])
    return n_ties


def _properties(g, T, V, min_obs):
    lh, vi, no, kp = g["lh"], g["vel_idx"], g["n_obs"], g["keep"]
    filled = vi >= 0
    # empty slots are exactly the documented empty value
    assert np.all(np.isneginf(lh[~filled])) and np.all(no[~filled] == 0)
    assert np.all(kp[~filled] == 0) and np.all(g["flux"][~filled] == 0)
    # filled slots: finite, valid index, enough usable epochs, keep bits < T
    assert np.all(np.isfinite(lh[filled])) and np.all(vi[filled] < V)
    assert np.all(no[filled] >= min_obs) and np.all(no[filled] <= T)
    if T < 64:
        assert np.all((kp[filled] >> np.uint64(T)) == 0)
    # best first, ties by smaller velocity index, empties last, no repeats
    a, b = lh[..., :-1], lh[..., 1:]
    ia, ib = vi[..., :-1], vi[..., 1:]
    ok = (a > b) | ((a == b) & (ia < ib)) | (ib < 0)
    assert np.all(ok | np.isneginf(a) & np.isneginf(b))
    assert np.all(~((ia < 0) & (ib >= 0)))


@pytest.fixture(scope="module")
def c2(kbm, oracle_mod):
    _say("full size: generating the DECam-CCD stack")
    st = synth.make_config(2)
    _say("full size: oracle planes")
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    psi, phi = psi.astype(np.float32), phi.astype(np.float32)
    p = dict(st.params)
    sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=True)
    item = dict(psi=torch.from_numpy(psi).cuda(), phi=torch.from_numpy(phi).cuda(),
                times=st.times, vels=st.vels, params=sp)
    _say("full size: batched persistent search (default schedule)")
    with kbm.BatchedSearch([item]) as plan:
        plan.run()
        assert not plan.check()
        g = _np(plan.results[0])
    del item
    torch.cuda.empty_cache()
    return st, psi, phi, p, g


def test_fullsize_c2_sampled_pixels(oracle_mod, c2):
    st, psi, phi, p, g = c2
    T, H, W = st.sci.shape
    rng = np.random.default_rng(7)
    pix = {(int(round(s["x0"])), int(round(s["y0"]))) for s in st.sources}
    pix |= {(int(x), int(y)) for x, y in zip(rng.integers(0, W, 60), rng.integers(0, H, 60))}
    pix |= {(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1), (W // 2, 0), (0, H // 2),
            (W - 1, H // 2), (W // 2, H - 1), (63, 17), (64, 17), (1983, 2048)}
    pix = sorted(pix)
    _say(f"full size: oracle on {len(pix)} sampled pixels")
    fp64 = {}
    ties = _pixel_check(oracle_mod, psi, phi, st, p, g, pix, fp64)
    _say(f"  near-tie swaps: {ties}")
    _say(f"  binary32 vs FP64 keep decisions: {fp64}")
    assert fp64["slots"] > 0
    # the injected sources are found at their start pixels
    hits = sum(int(g["lh"][int(round(s['y0'])), int(round(s['x0'])), 0] >= 10.0)
               for s in st.sources)
    _say(f"  sources with L' >= 10 at their start pixel: {hits}/{len(st.sources)}")
    assert hits >= 0.5 * len(st.sources)


def test_fullsize_c2_properties(c2):
    st, psi, phi, p, g = c2
    _properties(g, st.T, len(st.vels), p["min_obs"])


def test_fullsize_c5_sampled_pixels(kbm, oracle_mod):
    _say("full size: generating the full-pipeline stack")
    st = synth.make_config(5)
    _say("full size: oracle planes (T = 60)")
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    psi, phi = psi.astype(np.float32), phi.astype(np.float32)
    p = dict(st.params)
    sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=True)
    gpsi, gphi = torch.from_numpy(psi).cuda(), torch.from_numpy(phi).cuda()
    _say("full size: search (two plane descriptors)")
    g = _np(kbm.search(gpsi, gphi, st.times, st.vels, sp))
    del gpsi, gphi
    torch.cuda.empty_cache()
    T, H, W = st.sci.shape
    rng = np.random.default_rng(17)
    pix = {(int(round(s["x0"])), int(round(s["y0"]))) for s in st.sources[:40]}
    pix |= {(int(x), int(y)) for x, y in zip(rng.integers(0, W, 40), rng.integers(0, H, 40))}
    pix |= {(0, 0), (W - 1, H - 1), (W // 2, H // 2), (W - 1, 0), (0, H - 1)}
    _say(f"full size: oracle on {len(pix)} sampled pixels")
    fp64 = {}
    _pixel_check(oracle_mod, psi, phi, st, p, g, sorted(pix), fp64)
    _say(f"  binary32 vs FP64 keep decisions: {fp64}")
    _properties(g, T, len(st.vels), p["min_obs"])


def test_c3_recipe_batch(kbm, oracle_mod):
    specs = synth.make_batched_specs(62, sizes=(64, 96, 128, 160))
    items, stacks = [], []
    for sp_ in specs:
        st = synth.make_batched_stack(sp_, n_sources=2)
        psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
        psi, phi = psi.astype(np.float32), phi.astype(np.float32)
        p = dict(st.params)
        sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=True)
        items.append(dict(psi=torch.from_numpy(psi).cuda(), phi=torch.from_numpy(phi).cuda(),
                          times=st.times, vels=st.vels, params=sp))
        stacks.append((st, psi, phi, p))
    _say(f"c3 recipe: {len(items)} stacks, T {min(s['T'] for s in specs)}.."
         f"{max(s['T'] for s in specs)}, V {len(stacks[0][0].vels)}")
    with kbm.BatchedSearch(items) as plan:
        plan.run()
        assert not plan.check()
        res = [_np(r) for r in plan.results]
    rng = np.random.default_rng(11)
    for j, ((st, psi, phi, p), it, g) in enumerate(zip(stacks, items, res)):
        ref = kbm.search(it["psi"], it["phi"], it["times"], it["vels"], it["params"])
        r = _np(ref)
        for k in r:
            assert np.array_equal(r[k], g[k], equal_nan=True), (j, k)
        _properties(g, st.T, len(st.vels), p["min_obs"])
        H, W = st.H, st.W
        pix = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(3)]
        pix += [(int(round(s["x0"])), int(round(s["y0"]))) for s in st.sources]
        _pixel_check(oracle_mod, psi, phi, st, p, g, pix)


def _planes_window_check(oracle_mod, st, gpsi, gphi, x0, y0, w, h, terms_tol=1e-5):
    """Protocol A on a window: the oracle's planes of the images cropped
    with a margin of the PSF radius, compared on the window (whose pixels
    see every tap they would see in the full image)."""
    T, H, W = st.sci.shape
    r = st.psf.shape[0] // 2
    ya, yb = max(0, y0 - r), min(H, y0 + h + r)
    xa, xb = max(0, x0 - r), min(W, x0 + w + r)
    sl = (slice(None), slice(ya, yb), slice(xa, xb))
    sci, var = np.ascontiguousarray(st.sci[sl]), np.ascontiguousarray(st.var[sl])
    mask = np.ascontiguousarray(st.mask[sl])
    rpsi, rphi = oracle_mod.planes(sci, var, mask, st.psf)
    terms = P.plane_terms_abs(oracle_mod, sci, var, mask, st.psf)
    inner = (slice(None), slice(y0 - ya, y0 - ya + h), slice(x0 - xa, x0 - xa + w))
    gp = gpsi[:, y0:y0 + h, x0:x0 + w].cpu().numpy()
    gf = gphi[:, y0:y0 + h, x0:x0 + w].cpu().numpy()
    assert np.all(np.abs(gp - rpsi[inner]) <= terms_tol * terms[inner] + 1e-30)
    assert np.all(np.abs(gf - rphi[inner]) <= terms_tol * rphi[inner] + 1e-30)


def test_c3_fullsize_batch(kbm, oracle_mod):
    """The 62-stack batched workload at its full sides (512 .. 4096, T 10 ..
    30, 64 x 64 velocities, K = 8, sigma_G on) in one persistent launch:
    every stack's results bit-identical to its own per-stack search; planes
    against the oracle on windows (protocol A); sampled start pixels of
    every stack (random ones and injected sources) re-searched by the
    oracle on the same float32 planes (protocol B) with the keep decisions
    certified against the FP64 decision."""
    import concurrent.futures as cf
    specs = synth.make_batched_specs(62)
    rng = np.random.default_rng(62)
    items, meta = [], []
    _say(f"c3 full size: generating {len(specs)} stacks "
         f"({sum(s['W'] * s['H'] * s['T'] for s in specs) / 1e9:.2f}e9 pixel-epochs)")
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        for j, st in enumerate(ex.map(synth.make_batched_stack, specs)):
            sci, var = torch.from_numpy(st.sci).cuda(), torch.from_numpy(st.var).cuda()
            mask = torch.from_numpy(st.mask).cuda()
            psi, phi = kbm.make_planes(sci, var, mask, st.psf)
            del sci, var, mask
            T, H, W = st.sci.shape
            wx = (int(rng.integers(0, max(1, W - 48))), int(rng.integers(0, max(1, H - 40))))
            _planes_window_check(oracle_mod, st, psi, phi, wx[0], wx[1], min(48, W), min(40, H))
            _planes_window_check(oracle_mod, st, psi, phi, 0, H - 16, 16, 16)
            p = dict(st.params)
            sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=True)
            items.append(dict(psi=psi, phi=phi, times=st.times, vels=st.vels, params=sp))
            pix = [(int(rng.integers(0, W)), int(rng.integers(0, H))) for _ in range(2)]
            pix += [(int(round(s["x0"])), int(round(s["y0"]))) for s in st.sources[:2]]
            meta.append(dict(T=T, H=H, W=W, times=st.times, vels=st.vels, p=p, pix=pix,
                             sources=[dict(s) for s in st.sources]))
            del st
            if j % 8 == 7:
                _say(f"  {j + 1} stacks on the GPU, planes checked on windows")
    torch.cuda.synchronize()
    _say("c3 full size: one persistent launch over every stack")
    with kbm.BatchedSearch(items, want_lh_raw=False) as plan:
        plan.run()
        torch.cuda.synchronize()
        assert not plan.check()
        fp64 = {}
        ties = 0
        for j, (it, m, res) in enumerate(zip(items, meta, plan.results)):
            ref = kbm.search(it["psi"], it["phi"], it["times"], it["vels"], it["params"],
                             want_lh_raw=False)
            for key in ref:
                if ref[key] is not None:
                    assert torch.equal(ref[key], res[key]), (j, key)
            del ref
            g = _np(res)
            _properties(g, m["T"], len(m["vels"]), m["p"]["min_obs"])
            psi, phi = it["psi"].cpu().numpy(), it["phi"].cpu().numpy()

            class S:
                pass
            st = S()
            st.times, st.vels = m["times"], m["vels"]
            ties += _pixel_check(oracle_mod, psi, phi, st, m["p"], g, m["pix"], fp64)
            del psi, phi, g
            if j % 8 == 7:
                _say(f"  {j + 1} stacks: identical to per-stack, sampled pixels match")
    _say(f"  near-tie swaps {ties}; binary32 vs FP64 keep decisions: {fp64}")
    assert fp64["slots"] > 0
