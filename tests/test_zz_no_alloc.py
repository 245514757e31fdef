"""The allocation-free candidate extraction (kbm_extract_top_noalloc, for
callers that cannot allocate) gives exactly what kbm_extract_top gives.
Two calls in a row on one GPU, the second on a smaller input, so the shared
scratch holds the first call's contents when the second one starts; the
outputs are allocated once, by the caller, before either call."""
import ctypes as C

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


def _drawn_results(seed, Hr, Wr, K, V):
    """Result arrays drawn directly (ties, -inf and NaN included)."""
    rng = np.random.default_rng(seed)
    lh = rng.normal(size=(Hr, Wr, K)).round(2).astype(np.float32)
    lh[rng.random(lh.shape) < 0.1] = -np.inf
    lh.flat[5] = np.nan
    vidx = rng.integers(0, V, size=lh.shape).astype(np.int32)
    vidx[~np.isfinite(lh)] = -1
    cu = lambda a: torch.from_numpy(a).cuda()
    res = dict(lh=cu(lh), vel_idx=cu(vidx),
               flux=cu(rng.normal(size=lh.shape).astype(np.float32)),
               n_obs=cu(rng.integers(0, 30, size=lh.shape).astype(np.int16)),
               keep=cu(rng.integers(0, 2 ** 62, size=lh.shape).astype(np.int64)))
    vels = rng.uniform(-50, 50, size=(V, 2)).astype(np.float32)
    return res, vels


def _searched_results(kbm):
    st = synth.make_config(2, size=(150, 70), n_vel=(6, 8))
    cu = lambda a: torch.from_numpy(a).cuda()
    psi, phi = kbm.make_planes(cu(st.sci), cu(st.var), cu(st.mask), st.psf)
    res = kbm.search(psi, phi, st.times, st.vels,
                     kbm.SearchParams(k=4, min_obs=20, region=(5, 3, 145, 60)))
    return res, st.vels


def test_extract_noalloc_matches_extract_top(kbm):
    cap = 6000
    dev = torch.device("cuda")
    out = dict(params=torch.empty((cap, 4), dtype=torch.float32, device=dev),
               lh=torch.empty(cap, dtype=torch.float32, device=dev),
               flux=torch.empty(cap, dtype=torch.float32, device=dev),
               keep=torch.empty(cap, dtype=torch.int64, device=dev),
               index=torch.empty(cap, dtype=torch.int64, device=dev),
               n_obs=torch.empty(cap, dtype=torch.int16, device=dev))
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    big = _drawn_results(21, 300, 257, 8, 500)        # 616800 slots, 2410 blocks
    small = _drawn_results(22, 17, 29, 3, 40)         # 1479 slots, 6 blocks
    cases = [("large", big, 5000, -np.inf, (3, 7)),
             ("smaller", small, 300, 0.25, (0, 0)),
             ("searched", _searched_results(kbm), 200, -np.inf, (5, 3)),
             ("nothing qualifies", small, 50, 1e9, (0, 0))]
    for name, (res, vels), n_max, lh_min, origin in cases:
        print(f"extraction case {name}: n_max {n_max}", flush=True)
        ref = kbm.extract_top(res, vels, n_max, lh_min, region_origin=origin)
        vdev = torch.from_numpy(np.ascontiguousarray(vels)).cuda()
        kbm.extract_top_noalloc(res, vdev, n_max, out, n_out, lh_min, region_origin=origin)
        torch.cuda.synchronize()
        n = int(n_out.item())
        assert n == ref["lh"].numel(), (name, n, ref["lh"].numel())
        for key in ("params", "lh", "flux", "keep", "index", "n_obs"):
            assert torch.equal(out[key][:n], ref[key]), (name, key)


def test_extract_noalloc_rejects_bad_sizes(kbm):
    L = kbm.lib()
    fake = C.c_void_p(0x1000)   # never dereferenced: validation fails first
    r = kbm._Results(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, None)
    args = lambda Hr, Wr, k, nv, nmax: (C.byref(r), Hr, Wr, k, 0, 0, fake, nv, 0.0, nmax,
                                        fake, fake, None, None, None, None, fake, None)
    assert L.kbm_extract_top_noalloc(*args(65536, 65536, 1, 4, 10)) == 2   # 2^32 slots
    assert b"2^32" in L.kbm_last_error()
    assert L.kbm_extract_top_noalloc(*args(10, 10, 17, 4, 10)) == 1        # k > 16
    assert L.kbm_extract_top_noalloc(*args(10, 10, 2, 0, 10)) == 1         # no velocities
    assert L.kbm_extract_top_noalloc(*args(10, 10, 2, 4, -1)) == 1         # n_max < 0
