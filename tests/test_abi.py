"""The C ABI library loads without a GPU, exports every entry point that
include/kbm.h declares, and rejects bad arguments on the host before any
HIP call."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(kbm_\w+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    import paper_2109_03296_amd as kbm
    return kbm.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert {"kbm_make_planes", "kbm_search", "kbm_search_workspace_size",
            "kbm_sigmag_filter", "kbm_refine", "kbm_status_string",
            "kbm_last_error", "kbm_version"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_build_id_matches_sources(L):
    from paper_2109_03296_amd import build
    L.kbm_build_id.restype = C.c_char_p
    assert L.kbm_build_id().decode() == build.source_hash()


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    """A comment edit keeps the build id; code (even a '//' inside a string
    literal) and extra flags change it."""
    import shutil
    from paper_2109_03296_amd import build
    src = tmp_path / "csrc"
    shutil.copytree(build.CSRC, src)
    monkeypatch.setattr(build, "CSRC", str(src))
    h0 = build.source_hash()
    f = src / "sigmag.hip"
    f.write_text(f.read_text() + "\n// a new comment\n/* and\n another */\n")
    assert build.source_hash() == h0
    f.write_text(f.read_text() + 'static const char *s = "// not a comment";\n')
    assert build.source_hash() != h0
    assert build.source_hash(("-DX=1",)) != build.source_hash()


def test_status_strings(L):
    assert L.kbm_status_string(0) == b"ok"
    assert L.kbm_status_string(1) == b"invalid argument"
    assert L.kbm_status_string(5) == b"workspace too small"
    assert L.kbm_version() >= 100


def _stack(T=5, H=8, W=9, times=None):
    import paper_2109_03296_amd as kbm
    t = np.linspace(0, 1, T) if times is None else np.asarray(times, np.float64)
    return kbm._Stack(W, H, T, t.ctypes.data), t


FAKE = C.c_void_p(0x1000)   # never dereferenced: validation fails first


def test_make_planes_validation(L):
    st, t = _stack()
    psf = np.ones((3, 3), np.float32)
    pp = psf.ctypes.data_as(C.c_void_p)
    assert L.kbm_make_planes(None, FAKE, FAKE, None, pp, 3, FAKE, FAKE, None) == 1
    assert L.kbm_make_planes(C.byref(st), FAKE, FAKE, None, pp, 4, FAKE, FAKE, None) == 1
    assert b"odd" in L.kbm_last_error()
    big = np.ones((33, 33), np.float32)
    assert L.kbm_make_planes(C.byref(st), FAKE, FAKE, None,
                             big.ctypes.data_as(C.c_void_p), 33, FAKE, FAKE, None) == 2
    assert L.kbm_make_planes(C.byref(st), None, FAKE, None, pp, 3, FAKE, FAKE, None) == 1
    st65, t65 = _stack(T=65)
    assert L.kbm_make_planes(C.byref(st65), FAKE, FAKE, None, pp, 3, FAKE, FAKE, None) == 1
    stn, tn = _stack(times=[0.0, float("nan"), 1.0, 2.0, 3.0])
    assert L.kbm_make_planes(C.byref(stn), FAKE, FAKE, None, pp, 3, FAKE, FAKE, None) == 1
    assert b"not finite" in L.kbm_last_error()
    nanpsf = psf.copy()
    nanpsf[1, 1] = np.nan
    assert L.kbm_make_planes(C.byref(st), FAKE, FAKE, None,
                             nanpsf.ctypes.data_as(C.c_void_p), 3, FAKE, FAKE, None) == 1


def _params(vels, **kw):
    import paper_2109_03296_amd as kbm
    d = dict(k=4, min_obs=1, sigmag=1, q_lo=0.25, q_hi=0.75, coeff=0.7413,
             n_sigma=2.0, region=(0, 0, 9, 8))
    d.update(kw)
    x0, y0, x1, y1 = d["region"]
    return kbm._SearchParams(vels.ctypes.data, vels.shape[0], d["k"], d["min_obs"],
                             d["sigmag"], d["q_lo"], d["q_hi"], d["coeff"],
                             d["n_sigma"], x0, y0, x1, y1)


def test_search_validation_and_workspace_size(L):
    st, t = _stack()
    vels = np.array([[1.0, 2.0], [0.0, 0.0], [-3.0, 1.0]], np.float32)
    nb = C.c_size_t(0)
    p = _params(vels)
    assert L.kbm_search_workspace_size(C.byref(st), C.byref(p), 1, C.byref(nb)) == 0
    # packed (nu, s) planes, offset tables, flags, top-K state
    def up(x, a=256):
        return math.ceil(x / a) * a
    T, H, W, V, K = 5, 8, 9, 3, 4
    # off16, lin, per-velocity box + repeat counts (32 B), mbox (16 B), ranks
    tab = up(up(up(up(V * T * 4, 16) + V * T * 4, 32) + V * 32, 16) + V * 16, 16) + 3 * 65 * 4
    pk = up(T * H * W * 8)
    flags = up(pk + tab)
    stl = up(flags + 256)
    sti = up(stl + 4 * H * W * K)
    assert nb.value == up(sti + 4 * H * W * K)
    for bad in (dict(k=0), dict(k=17), dict(min_obs=0), dict(sigmag=2),
                dict(q_lo=0.8), dict(q_hi=1.5), dict(coeff=-1.0),
                dict(n_sigma=float("nan")), dict(region=(0, 0, 10, 8)),
                dict(region=(5, 0, 4, 8))):
        pb = _params(vels, **bad)
        assert L.kbm_search_workspace_size(C.byref(st), C.byref(pb), 1,
                                           C.byref(nb)) == 1, bad
    nanv = np.array([[np.nan, 1.0]], np.float32)
    pn = _params(nanv)
    assert L.kbm_search_workspace_size(C.byref(st), C.byref(pn), 1, C.byref(nb)) == 1
    # undersized workspace is reported before anything is enqueued
    import paper_2109_03296_amd as kbm
    planes = (C.c_void_p * 1)(0x1000)
    res = (kbm._Results * 1)(kbm._Results(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, None))
    rc = L.kbm_search(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE,
                      C.c_size_t(16), None)
    assert rc == 5 and b"workspace" in L.kbm_last_error()
    assert L.kbm_search(C.byref(st), planes, planes, C.byref(p), res, 0, FAKE,
                        C.c_size_t(1 << 30), None) == 1


def test_batch_validation(L):
    import paper_2109_03296_amd as kbm
    st, t = _stack()
    vels = np.array([[1.0, 2.0], [0.0, 0.0], [-3.0, 1.0]], np.float32)
    p = _params(vels)
    nb, ns = C.c_size_t(0), C.c_size_t(0)
    assert L.kbm_batch_workspace_size(C.byref(st), C.byref(p), 1, C.byref(nb)) == 0
    assert L.kbm_search_workspace_size(C.byref(st), C.byref(p), 1, C.byref(ns)) == 0
    assert nb.value > ns.value   # per-stack blocks plus queues and counters
    # beyond the persistent kernel's limits: unsupported (kbm_search covers it)
    st33, t33 = _stack(T=33)
    assert L.kbm_batch_workspace_size(C.byref(st33), C.byref(p), 1, C.byref(nb)) == 2
    p9 = _params(vels, k=9)
    assert L.kbm_batch_workspace_size(C.byref(st), C.byref(p9), 1, C.byref(nb)) == 2
    assert L.kbm_batch_workspace_size(C.byref(st), C.byref(p), 0, C.byref(nb)) == 1
    planes = (C.c_void_p * 1)(0x1000)
    res = (kbm._Results * 1)(kbm._Results(0x1000, 0x1000, 0x1000, 0x1000, 0x1000, None))
    h = C.c_void_p()
    big = C.c_size_t(1 << 30)
    # bad tune mode, bad given schedules, NULL handle, small workspace
    assert L.kbm_batch_create(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE, big,
                              7, None, None, C.byref(h)) == 1
    assert L.kbm_batch_create(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE, big,
                              2, None, None, C.byref(h)) == 1
    for bad in (dict(vel_block=16), dict(tile_cols=3), dict(tile_rows=128),
                dict(waves=2), dict(blocks_per_cu=-1), dict(sweep=2)):
        sc = kbm.Schedule(256, 4, 16, 1, 0, 0, 0.0)
        for f, v in bad.items():
            setattr(sc, f, v)
        assert L.kbm_batch_create(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE,
                                  big, 2, C.byref(sc), None, C.byref(h)) == 1, bad
    assert L.kbm_batch_create(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE, big,
                              0, None, None, None) == 1
    assert L.kbm_batch_create(C.byref(st), planes, planes, C.byref(p), res, 1, FAKE,
                              C.c_size_t(16), 0, None, None, C.byref(h)) == 5
    assert h.value is None
    assert L.kbm_batch_run(None, None) == 1
    stalled = C.c_int32(0)
    assert L.kbm_batch_check(None, None, C.byref(stalled)) == 1
    assert L.kbm_batch_destroy(None) == 0


def test_sigmag_and_refine_validation(L):
    assert L.kbm_sigmag_filter(FAKE, None, None, 10, 0, 0.25, 0.75, 0.7413, 2.0,
                               FAKE, None, None) == 1
    assert L.kbm_sigmag_filter(FAKE, None, None, 10, 65, 0.25, 0.75, 0.7413, 2.0,
                               FAKE, None, None) == 1
    assert L.kbm_sigmag_filter(None, None, None, 10, 5, 0.25, 0.75, 0.7413, 2.0,
                               FAKE, None, None) == 1
    assert L.kbm_sigmag_filter(FAKE, None, None, 10, 5, 0.75, 0.25, 0.7413, 2.0,
                               FAKE, None, None) == 1
    # nothing to do is not an error and touches no device
    assert L.kbm_sigmag_filter(None, None, None, 0, 5, 0.25, 0.75, 0.7413, 2.0,
                               None, None, None) == 0
    st, t = _stack()
    assert L.kbm_refine(C.byref(st), FAKE, FAKE, -1, FAKE, None, FAKE, None,
                        None, None, None, None) == 1
    assert L.kbm_refine(C.byref(st), FAKE, FAKE, 4, FAKE, None, FAKE, FAKE,
                        None, None, None, None) == 1
    assert L.kbm_refine(C.byref(st), None, None, 0, None, None, None, None,
                        None, None, None, None) == 0


def test_score_validation(L):
    st, t = _stack()
    args = lambda n, mo=1, sg=1, ql=0.25: (C.byref(st), FAKE, FAKE, n, FAKE, mo, sg, ql, 0.75,
                                           0.7413, 2.0, FAKE, FAKE, FAKE, FAKE, None, None)
    assert L.kbm_score_trajectories(*args(-1)) == 1
    assert L.kbm_score_trajectories(*args(4, mo=0)) == 1
    assert L.kbm_score_trajectories(*args(4, sg=2)) == 1
    assert L.kbm_score_trajectories(*args(4, ql=0.9)) == 1
    assert L.kbm_score_trajectories(*args(0)) == 0   # nothing to do, no device
    bad, tb = _stack(T=0)
    assert L.kbm_score_trajectories(C.byref(bad), FAKE, FAKE, 4, FAKE, 1, 1, 0.25, 0.75,
                                    0.7413, 2.0, FAKE, FAKE, FAKE, FAKE, None, None) == 1


def test_stamps_validation(L):
    st, t = _stack()
    a = lambda n, r=10, lim=None: (C.byref(st), FAKE, FAKE, None, n, FAKE, None, r, lim,
                                   None, FAKE, FAKE, None)
    assert L.kbm_stamps(*a(-1)) == 1
    assert L.kbm_stamps(*a(3, r=0)) == 1
    assert L.kbm_stamps(*a(3, r=16)) == 1
    bad = (C.c_double * 5)(0.5, float("nan"), 1.5, 36.5, 36.5)
    assert L.kbm_stamps(*a(3, lim=bad)) == 1
    assert L.kbm_stamps(*a(0)) == 0
    odd = C.c_void_p(0x1004)   # params must be 16-byte aligned
    assert L.kbm_stamps(C.byref(st), FAKE, FAKE, None, 3, odd, None, 10, None, None,
                        FAKE, FAKE, None) == 1


def test_sigmag_coeff_host(L):
    """C of Eq. 3 computed by the library on the host (no GPU needed)
    against scipy's normal quantiles."""
    from scipy import stats
    c = C.c_double(0.0)
    for ql, qh in ((0.25, 0.75), (0.1, 0.9), (0.05, 0.6), (0.3, 0.99)):
        assert L.kbm_sigmag_coeff(ql, qh, C.byref(c)) == 0
        want = 1.0 / (stats.norm.ppf(qh) - stats.norm.ppf(ql))
        assert c.value == pytest.approx(want, rel=1e-13)
    for ql, qh in ((0.0, 0.75), (0.5, 0.5), (0.2, 1.0), (float("nan"), 0.7)):
        assert L.kbm_sigmag_coeff(ql, qh, C.byref(c)) == 1
    assert L.kbm_sigmag_filter_ex(FAKE, None, None, 10, 5, 2, 0.25, 0.75, 0.7413, 2.0,
                                  0.0, FAKE, None, None, None) == 1
    assert L.kbm_sigmag_filter_ex(FAKE, None, None, 10, 5, 0, 0.25, 0.75, 0.7413, 2.0,
                                  float("nan"), FAKE, None, None, None) == 1


def test_binding_rejects_host_tensors():
    import torch
    import paper_2109_03296_amd as kbm
    x = torch.zeros(2, 4, 4)
    with pytest.raises(TypeError):
        kbm.make_planes(x, x, None, np.ones((3, 3), np.float32))


def test_detect_validation(L):
    L.kbm_detect.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                             C.c_float, C.c_void_p, C.c_void_p]
    assert L.kbm_detect(-1, FAKE, FAKE, FAKE, 1, 10.0, FAKE, None) == 1
    assert L.kbm_detect(5, None, FAKE, FAKE, 1, 10.0, FAKE, None) == 1
    assert L.kbm_detect(5, FAKE, FAKE, FAKE, 1, float("nan"), FAKE, None) == 1
    assert L.kbm_detect(0, None, None, None, 1, 10.0, None, None) == 0
