"""GPU parity: the HIP path (through the C ABI binding) against the FP64
oracle on the same seeded inputs.

Protocol A: GPU planes vs oracle planes.
Protocol B: both searches read the oracle's planes rounded to float32, so
            keep masks must be bit-identical and top-K identical up to near
            ties.
Protocol C: each side builds its own planes from the images.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from tests import parity as P

pytestmark = pytest.mark.gpu


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


def _cuda(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _oracle_planes32(oracle_mod, st):
    psi, phi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    return psi.astype(np.float32), phi.astype(np.float32)


def _single_eval(oracle_mod, psi, phi, st, region, p):
    x0, y0 = region[0], region[1]

    def f(y, x, v):
        o = oracle_mod.search(psi, phi, st.times, st.vels[v:v + 1], k=1,
                              region=(x0 + x, y0 + y, x0 + x + 1, y0 + y + 1),
                              **{k: p[k] for k in ("min_obs", "sigmag", "q_lo",
                                                   "q_hi", "coeff", "n_sigma")})
        return float(o["lh"][0, 0, 0])
    return f


# ---------------------------------------------------------------- planes --
@pytest.mark.parametrize("case", ["c1", "c2crop", "tiny_nan", "c5crop"])
def test_planes_protocol_A(kbm, oracle_mod, case):
    _say(f"planes protocol A: {case}")
    if case == "c1":
        st = synth.make_config(1)
    elif case == "c2crop":
        st = synth.make_config(2, size=(300, 200), n_vel=(4, 4))
    elif case == "c5crop":
        st = synth.make_config(5, size=(130, 97), n_vel=(4, 4))
    else:
        st = synth.tiny_stack(3, W=37, H=29, T=7, k=5, mask_rate=0.2,
                              masked_fill=np.nan)
    psi, phi = kbm.make_planes(_cuda(st.sci), _cuda(st.var), _cuda(st.mask),
                               st.psf)
    rpsi, rphi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    terms = P.plane_terms_abs(oracle_mod, st.sci, st.var, st.mask, st.psf)
    gpsi, gphi = psi.cpu().numpy(), phi.cpu().numpy()
    assert np.all(np.abs(gpsi - rpsi) <= 1e-5 * terms + 1e-30)
    assert np.all(np.abs(gphi - rphi) <= 1e-5 * rphi + 1e-30)


def _rotated_psf(k, sx=1.8, sy=0.9, theta=0.6):
    """Elliptical Gaussian rotated off the axes: not an outer product."""
    r = k // 2
    y, x = np.mgrid[-r:r + 1, -r:r + 1].astype(np.float64)
    u = np.cos(theta) * x + np.sin(theta) * y
    v = -np.sin(theta) * x + np.cos(theta) * y
    g = np.exp(-0.5 * (u * u / (sx * sx) + v * v / (sy * sy)))
    return (g / g.sum()).astype(np.float32)


@pytest.mark.parametrize("psf_case", ["rotated9", "gauss25", "delta1", "gauss_rowzero",
                                      "gauss31", "rotated31"])
def test_planes_psf_shapes(kbm, oracle_mod, psf_case):
    """Rank-1 PSFs take the two-pass kernel, others the direct one (a
    direct PSF wider than 25 in two launches over row ranges); all meet the
    same bound against the oracle, on a ragged 3-tile x 3-tile image."""
    _say(f"planes psf shapes: {psf_case}")
    st = synth.tiny_stack(11, W=150, H=37, T=3, k=5, mask_rate=0.1)
    if psf_case == "rotated9":
        st.psf = _rotated_psf(9)
    elif psf_case == "gauss25":
        st.psf = synth.gaussian_psf(3.0, 25)
    elif psf_case == "gauss31":
        st.psf = synth.gaussian_psf(4.0, 31)
    elif psf_case == "rotated31":   # direct kernel over two row ranges
        st.psf = _rotated_psf(31, sx=5.0, sy=2.5)
    elif psf_case == "delta1":
        st.psf = np.ones((1, 1), np.float32)
    else:
        g = synth.gaussian_psf(1.2, 7).astype(np.float64)
        g[0, :] = 0.0      # still an outer product, with a zero factor entry
        st.psf = (g / g.sum()).astype(np.float32)
    psi, phi = kbm.make_planes(_cuda(st.sci), _cuda(st.var), _cuda(st.mask), st.psf)
    rpsi, rphi = oracle_mod.planes(st.sci, st.var, st.mask, st.psf)
    terms = P.plane_terms_abs(oracle_mod, st.sci, st.var, st.mask, st.psf)
    gpsi, gphi = psi.cpu().numpy(), phi.cpu().numpy()
    assert np.all(np.abs(gpsi - rpsi) <= 1e-5 * terms + 1e-30)
    assert np.all(np.abs(gphi - rphi) <= 1e-5 * rphi + 1e-30)


def test_planes_separable_matches_direct(kbm):
    """The same Gaussian through both kernels: a perturbation of one tap by
    1e-4 of the peak (well above the rank-1 test's 1e-6) sends it to the
    direct kernel; the results agree to the size of that perturbation."""
    st = synth.tiny_stack(12, W=130, H=50, T=4, k=9, mask_rate=0.1)
    g = st.psf.copy()
    h = g.copy()
    h[0, 0] += np.float32(1e-4) * g.max()
    a = kbm.make_planes(_cuda(st.sci), _cuda(st.var), _cuda(st.mask), g)
    b = kbm.make_planes(_cuda(st.sci), _cuda(st.var), _cuda(st.mask), h)
    scale = float(torch.max(torch.abs(a[0])))
    assert float(torch.max(torch.abs(a[0] - b[0]))) < 1e-3 * scale
    assert not torch.equal(a[0], b[0])


def test_planes_masked_fill_bitwise(kbm):
    a = synth.tiny_stack(4, W=70, H=33, T=5, k=7, mask_rate=0.3)
    b = synth.tiny_stack(4, W=70, H=33, T=5, k=7, mask_rate=0.3, masked_fill=1e30)
    pa = kbm.make_planes(_cuda(a.sci), _cuda(a.var), _cuda(a.mask), a.psf)
    pb = kbm.make_planes(_cuda(b.sci), _cuda(b.var), _cuda(b.mask), b.psf)
    assert torch.equal(pa[0], pb[0]) and torch.equal(pa[1], pb[1])


# ---------------------------------------------------------------- search --
def _slow(st):
    """T = 60 over 4 days: a slow grid keeps tracks inside a small crop."""
    import math
    st.vels = synth.velocity_grid(np.linspace(0.0, 22.0, 10),
                                  np.linspace(-math.pi, math.pi, 12, endpoint=False))
    return st


SEARCH_CASES = {
    # name: (stack factory, param overrides, region)
    "c1": (lambda: synth.make_config(1), {}, None),
    "c2crop_sg": (lambda: synth.make_config(2, size=(300, 200), n_vel=(16, 24)),
                  {}, None),
    "c2crop_plain_k16": (lambda: synth.make_config(2, size=(300, 200), n_vel=(12, 12)),
                         dict(sigmag=0, k=16), (5, 3, 290, 150)),
    "c5crop": (lambda: _slow(synth.make_config(5, size=(160, 128), n_vel=(4, 4))),
               dict(k=8), None),
    "tiny_t4": (lambda: synth.tiny_stack(11, W=70, H=9, T=4, n_vel=23), dict(k=5), None),
    "tiny_t17": (lambda: synth.tiny_stack(12, W=33, H=21, T=17, n_vel=19,
                                          max_speed=9.0), dict(k=3, min_obs=5), None),
    "tiny_t40": (lambda: synth.tiny_stack(13, W=65, H=12, T=40, n_vel=9,
                                          mask_rate=0.3), dict(k=4, min_obs=10), None),
    "tiny_t64": (lambda: synth.tiny_stack(14, W=20, H=18, T=64, n_vel=7),
                 dict(k=2, min_obs=1, n_sigma=1.0), None),
    # other percentile pairs take the runtime-rank path of the fused filter
    "c2crop_q16_84": (lambda: synth.make_config(2, size=(300, 200), n_vel=(12, 16)),
                      dict(q_lo=0.16, q_hi=0.84, coeff=0.5035), None),
    "tiny_t17_q10_90": (lambda: synth.tiny_stack(17, W=33, H=21, T=17, n_vel=19,
                                                 max_speed=9.0, mask_rate=0.1),
                        dict(k=3, min_obs=5, q_lo=0.1, q_hi=0.9, coeff=0.39,
                             n_sigma=3.0), None),
}


def _search_both(kbm, oracle_mod, st, over, region, protocol="B"):
    p = dict(st.params)
    p.update(over)
    H, W = st.H, st.W
    reg = region or (0, 0, W, H)
    psi, phi = _oracle_planes32(oracle_mod, st)
    if protocol == "B":
        gpsi, gphi = _cuda(psi), _cuda(phi)
    else:
        gpsi, gphi = kbm.make_planes(_cuda(st.sci), _cuda(st.var),
                                     _cuda(st.mask), st.psf)
    sp = kbm.SearchParams(k=p["k"], min_obs=p["min_obs"], sigmag=bool(p["sigmag"]),
                          q_lo=p["q_lo"], q_hi=p["q_hi"], coeff=p["coeff"],
                          n_sigma=p["n_sigma"], region=reg)
    g = kbm.search(gpsi, gphi, st.times, st.vels, sp)
    torch.cuda.synchronize()
    r = oracle_mod.search(psi, phi, st.times, st.vels, region=reg, **p)
    return g, r, psi, phi, p, reg


@pytest.mark.parametrize("name", list(SEARCH_CASES))
def test_search_protocol_B(kbm, oracle_mod, name):
    make, over, region = SEARCH_CASES[name]
    st = make()
    _say(f"search protocol B: {name} T={st.T} H={st.H} W={st.W} V={len(st.vels)}")
    g, r, psi, phi, p, reg = _search_both(kbm, oracle_mod, st, over, region)
    stats = P.compare_search(g, r, _single_eval(oracle_mod, psi, phi, st, reg, p))
    _say(f"  {stats}")
    gn = P.to_np(g)
    assert np.any(gn["vel_idx"] >= 0)
    if p["sigmag"]:
        # the binary32 keep decisions against the FP64 decision (Eqs. 1-5)
        cert = P.certify_fp64(oracle_mod, gn, psi, phi, st.times, st.vels, p, reg)
        _say(f"  FP64 decision: {cert}")


def test_search_duplicate_velocities_tie_rule(kbm, oracle_mod):
    st = synth.tiny_stack(15, W=40, H=11, T=6, n_vel=6)
    st.vels = np.concatenate([st.vels, st.vels[::-1], np.zeros((3, 2), np.float32)])
    g, r, psi, phi, p, reg = _search_both(kbm, oracle_mod, st, dict(k=8), None)
    stats = P.compare_search(g, r, None)   # exact ties: identical choices
    assert stats["tie_swaps"] == 0


def test_search_deterministic(kbm, oracle_mod):
    st = synth.make_config(2, size=(200, 130), n_vel=(8, 8))
    psi, phi = _oracle_planes32(oracle_mod, st)
    a = kbm.search(_cuda(psi), _cuda(phi), st.times, st.vels, k=8, min_obs=20)
    b = kbm.search(_cuda(psi), _cuda(phi), st.times, st.vels, k=8, min_obs=20)
    for key in a:
        if a[key] is not None:
            assert torch.equal(a[key], b[key]), key


def test_search_empty_and_all_masked(kbm, oracle_mod):
    st = synth.tiny_stack(16, W=30, H=10, T=5, n_vel=4)
    psi = _cuda(np.zeros((5, 10, 30), np.float32))
    phi = _cuda(np.zeros((5, 10, 30), np.float32))
    out = kbm.search(psi, phi, st.times, st.vels, k=3)
    torch.cuda.synchronize()
    o = P.to_np(out)
    assert np.all(o["vel_idx"] == -1) and np.all(np.isneginf(o["lh"]))
    assert np.all(o["keep"] == 0) and np.all(o["n_obs"] == 0)
    e = kbm.search(psi, phi, st.times, st.vels, k=3, region=(4, 4, 4, 9))
    assert e["lh"].shape == (5, 0, 3)


@pytest.mark.parametrize("name", ["c2crop", "c5crop"])
def test_search_protocol_C(kbm, oracle_mod, name):
    """End to end from the images: each side builds its own planes, which
    differ by rounding.  Every GPU slot is explained by the oracle: equal
    keep masks with L' within 1e-4, or keep flips whose FP64 decision margin
    lies within the plane-error bound of protocol A (certified); velocity
    swaps are near ties or carry such a certified flip."""
    if name == "c2crop":
        st = synth.make_config(2, size=(260, 190), n_vel=(12, 16))
    else:
        st = _slow(synth.make_config(5, size=(150, 120), n_vel=(4, 4)))
    _say(f"search protocol C: {name}")
    g, r, psi, phi, p, reg = _search_both(kbm, oracle_mod, st, {}, None, protocol="C")
    gpsi, gphi = kbm.make_planes(_cuda(st.sci), _cuda(st.var), _cuda(st.mask), st.psf)
    terms = P.plane_terms_abs(oracle_mod, st.sci, st.var, st.mask, st.psf)
    sp = kbm.SearchParams(k=1, min_obs=p["min_obs"], sigmag=bool(p["sigmag"]),
                          q_lo=p["q_lo"], q_hi=p["q_hi"], coeff=p["coeff"],
                          n_sigma=p["n_sigma"])

    def gpu_eval(x, y, v):
        prm = torch.tensor([[x, y, float(st.vels[v, 0]), float(st.vels[v, 1])]],
                           dtype=torch.float32, device="cuda")
        o = kbm.score_trajectories(gpsi, gphi, st.times, prm, sp)
        return (int(o["keep"].cpu().numpy().view(np.uint64)[0]),
                float(o["lh"].cpu().numpy()[0]))

    stats = P.compare_protocol_c(oracle_mod, g, r, psi, phi, terms, st.times, st.vels,
                                 p, gpu_eval, reg)
    _say(f"  {stats}")
    assert stats["slots"] > 0


# ---------------------------------------------------------------- sigma_G --
@pytest.mark.parametrize("T", [1, 2, 5, 26, 33, 60, 64])
def test_sigmag_filter(kbm, oracle_mod, T):
    rng = np.random.default_rng(100 + T)
    n = 3000
    ps = rng.standard_t(3, size=(n, T)).astype(np.float32)
    ph = rng.uniform(0.1, 3.0, size=(n, T)).astype(np.float32)
    valid = (rng.random((n, T)) > 0.15).astype(np.uint8)
    ph[rng.random((n, T)) < 0.02] = 0.0
    ps[:50] = 3.25                             # constant lightcurves
    for phi_given in (True, False):
        k_g, l_g = kbm.sigmag_filter(_cuda(ps), _cuda(ph) if phi_given else None,
                                     _cuda(valid))
        k_r, l_r = oracle_mod.sigmag(ps, ph if phi_given else None, valid)
        kg = k_g.cpu().numpy().view(np.uint64)
        assert np.array_equal(kg, k_r)
        assert np.all(P.lh_close(l_g.cpu().numpy(), l_r))
        # against the FP64 decision: differing bits lie within binary32
        # rounding of the threshold
        k64, _, mg, numax = oracle_mod.sigmag(ps, ph if phi_given else None, valid,
                                              decision="f64", want_margin=True)
        bits = P._bits(kg ^ k64, T)
        bound = P.f32_margin_bound(numax)[:, None]
        assert np.all(np.abs(mg[bits]) <= np.broadcast_to(bound, mg.shape)[bits])
        _say(f"  T={T} phi={phi_given}: {int(bits.sum())} keep bits differ from "
             f"the FP64 decision, all within the binary32 bound")


@pytest.mark.parametrize("T", [3, 26, 33])
def test_sigmag_filter_unaligned_inputs(kbm, T):
    """Arrays that do not start on a 16-byte boundary take the element-wise
    staging path; its results equal the 16-byte path's bit for bit, for
    ragged counts and partial last workgroups."""
    rng = np.random.default_rng(7 + T)
    for n in (1, 63, 65, 1000):
        ps = rng.standard_t(3, size=(n, T)).astype(np.float32)
        ph = rng.uniform(0.1, 3.0, size=(n, T)).astype(np.float32)
        valid = (rng.random((n, T)) > 0.15).astype(np.uint8)
        k_a, l_a = kbm.sigmag_filter(_cuda(ps), _cuda(ph), _cuda(valid))
        # views one element into larger buffers: 4-byte and 1-byte offsets
        fb = torch.zeros(n * T + 1, dtype=torch.float32, device="cuda")
        gb = torch.zeros(n * T + 1, dtype=torch.float32, device="cuda")
        vb = torch.zeros(n * T + 1, dtype=torch.uint8, device="cuda")
        fb[1:] = _cuda(ps).reshape(-1)
        gb[1:] = _cuda(ph).reshape(-1)
        vb[1:] = _cuda(valid).reshape(-1)
        psv, phv, vv = fb[1:].view(n, T), gb[1:].view(n, T), vb[1:].view(n, T)
        assert psv.data_ptr() % 16 != 0 and vv.data_ptr() % 16 != 0
        k_u, l_u = kbm.sigmag_filter(psv, phv, vv)
        assert torch.equal(k_u, k_a)
        assert torch.equal(l_u.view(torch.int32), l_a.view(torch.int32))


# ---------------------------------------------------------------- refine --
def _refine_setup(oracle_mod, n=2000, seed=5):
    st = synth.make_config(2, size=(256, 192), n_vel=(4, 4))
    psi, phi = _oracle_planes32(oracle_mod, st)
    rng = np.random.default_rng(seed)
    params = np.stack([rng.uniform(-5, 260, n), rng.uniform(-5, 195, n),
                       rng.uniform(-60, 60, n), rng.uniform(-40, 40, n)],
                      axis=1).astype(np.float32)
    keep = rng.integers(0, 2 ** 26, size=n).astype(np.uint64)
    return st, psi, phi, params, keep


def test_refine_forward_and_gradient(kbm, oracle_mod):
    st, psi, phi, params, keep = _refine_setup(oracle_mod)
    g_up = np.random.default_rng(9).normal(size=len(params)).astype(np.float32)
    gpsi = torch.zeros(psi.shape, device="cuda")
    gphi = torch.zeros(phi.shape, device="cuda")
    lh, gp = kbm.refine_backward(_cuda(psi), _cuda(phi), st.times, _cuda(params),
                                 _cuda(g_up), _cuda(keep.view(np.int64)),
                                 gpsi, gphi)
    rl, rg, rpsi, rphi = oracle_mod.refine(psi, phi, st.times, params, keep,
                                           grad_lh=g_up.astype(np.float64),
                                           want_planes=True)
    assert np.all(P.lh_close(lh.cpu().numpy(), rl))
    gpn = gp.cpu().numpy().astype(np.float64)
    num = np.linalg.norm(gpn - rg, axis=1)
    den = np.linalg.norm(rg, axis=1)
    big = den > 1e-3 * np.median(den[den > 0])
    assert np.all(num[big] <= 1e-4 * den[big] + 1e-6)
    scale = np.abs(rpsi).max()
    assert np.allclose(gpsi.cpu().numpy(), rpsi, rtol=1e-4, atol=1e-5 * scale)
    scale = np.abs(rphi).max()
    assert np.allclose(gphi.cpu().numpy(), rphi, rtol=1e-4, atol=1e-5 * scale)
    lf = kbm.refine_forward(_cuda(psi), _cuda(phi), st.times, _cuda(params),
                            _cuda(keep.view(np.int64)))
    assert torch.equal(lf, lh)


def test_refine_fd_fp32_and_autograd(kbm, oracle_mod):
    st, psi, phi, params, _ = _refine_setup(oracle_mod, n=300, seed=6)
    P_ = _cuda(params).requires_grad_(True)
    gpsi_t, gphi_t = _cuda(psi), _cuda(phi)
    L = kbm.TrajLH.apply(P_, gpsi_t, gphi_t, st.times, None)
    L.sum().backward()
    g = P_.grad.cpu().numpy()
    _, rg = oracle_mod.refine(psi, phi, st.times, params, None,
                              grad_lh=np.ones(len(params)))
    den = np.linalg.norm(rg, axis=1)
    big = den > 1e-3 * np.median(den[den > 0])
    assert np.all(np.linalg.norm(g - rg, axis=1)[big] <= 1e-4 * den[big] + 1e-6)
    # fp32 central differences, h = 1e-3 (smoke-level agreement)
    h = 1e-3
    fd = np.zeros_like(g)
    for j in range(4):
        pp, pm = params.copy(), params.copy()
        pp[:, j] += h
        pm[:, j] -= h
        lp = kbm.refine_forward(gpsi_t, gphi_t, st.times, _cuda(pp)).cpu().numpy()
        lm = kbm.refine_forward(gpsi_t, gphi_t, st.times, _cuda(pm)).cpu().numpy()
        fd[:, j] = (lp.astype(np.float64) - lm) / (pp[:, j].astype(np.float64) - pm[:, j])
    rel = np.linalg.norm(fd - g, axis=1) / np.maximum(np.linalg.norm(g, axis=1), 1e-3)
    assert np.median(rel) < 1e-2


def test_trajlh_plane_gradients_through_autograd(kbm, oracle_mod):
    """TrajLH with psi and phi requiring grad: autograd returns the adjoint's
    parameter gradient and its scatter-added plane gradients, both against
    the FP64 oracle (upstream gradient of a weighted sum, keep masks given)."""
    st, psi, phi, params, keep = _refine_setup(oracle_mod, n=400, seed=12)
    w = np.random.default_rng(13).normal(size=len(params))
    P_ = _cuda(params).requires_grad_(True)
    psi_t = _cuda(psi).requires_grad_(True)
    phi_t = _cuda(phi).requires_grad_(True)
    L = kbm.TrajLH.apply(P_, psi_t, phi_t, st.times, _cuda(keep.view(np.int64)))
    (L * _cuda(w.astype(np.float32))).sum().backward()
    rl, rg, rpsi, rphi = oracle_mod.refine(psi, phi, st.times, params, keep,
                                           grad_lh=w.astype(np.float32).astype(np.float64),
                                           want_planes=True)
    assert np.all(P.lh_close(L.detach().cpu().numpy(), rl))
    g = P_.grad.cpu().numpy().astype(np.float64)
    den = np.linalg.norm(rg, axis=1)
    big = den > 1e-3 * np.median(den[den > 0])
    assert np.all(np.linalg.norm(g - rg, axis=1)[big] <= 1e-4 * den[big] + 1e-6)
    for got, want in ((psi_t.grad, rpsi), (phi_t.grad, rphi)):
        scale = np.abs(want).max()
        assert scale > 0
        assert np.allclose(got.cpu().numpy(), want, rtol=1e-4, atol=1e-5 * scale)


def test_refine_graph_and_fused_match_eager(kbm, oracle_mod):
    """The refinement loop replayed from its captured graph, and the whole
    loop run by one fused kernel launch, give bit for bit what the eager
    launches give: several replays with other inputs and eager work between
    them, with and without keep masks."""
    st, psi, phi, params, keep = _refine_setup(oracle_mod, n=700, seed=14)
    gpsi, gphi = _cuda(psi), _cuda(phi)
    rng = np.random.default_rng(15)
    r = kbm.Refiner(gpsi, gphi, st.times, len(params), with_keep=True, steps=20)
    r0 = kbm.Refiner(gpsi, gphi, st.times, len(params), steps=20)
    for rep in range(3):
        p0 = params + rng.normal(scale=0.3, size=params.shape).astype(np.float32)
        k0 = _cuda(keep.view(np.int64))
        pe, le = kbm.refine(gpsi, gphi, st.times, _cuda(p0), k0, steps=20, mode="eager")
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        pg, lg = r.run(_cuda(p0), k0)
        torch.cuda.synchronize()
        assert torch.equal(pg, pe) and torch.equal(lg, le), rep
        pe, le = kbm.refine(gpsi, gphi, st.times, _cuda(p0), None, steps=20, mode="eager")
        pg, lg = r0.run(_cuda(p0))
        torch.cuda.synchronize()
        assert torch.equal(pg, pe) and torch.equal(lg, le), rep
        del junk
    for keep_t in (None, _cuda(keep.view(np.int64))):
        pe, le = kbm.refine(gpsi, gphi, st.times, _cuda(params), keep_t, steps=20,
                            mode="eager")
        for mode in ("graph", "fused"):
            pm, lm = kbm.refine(gpsi, gphi, st.times, _cuda(params), keep_t, steps=20,
                                mode=mode)
            torch.cuda.synchronize()
            assert torch.equal(pm, pe) and torch.equal(lm, le), mode
    # the default (50 steps, fused) against the eager loop
    pd, ld = kbm.refine(gpsi, gphi, st.times, _cuda(params))
    pe, le = kbm.refine(gpsi, gphi, st.times, _cuda(params), mode="eager")
    assert torch.equal(pd, pe) and torch.equal(ld, le)


@pytest.mark.parametrize("quantity,ql,qh", [(1, 0.25, 0.75), (0, 0.1, 0.9), (1, 0.16, 0.84)])
def test_sigmag_filter_variants(kbm, oracle_mod, quantity, ql, qh):
    """Flux quantity, other quantile pairs with C of Eq. 3, and the ΣLH'
    post-filter flag: keep masks bit-identical to the oracle."""
    rng = np.random.default_rng(90 + quantity)
    n, T = 20000, 26
    ps = rng.normal(0, 3, (n, T)).astype(np.float32)
    ps[:, 5] += rng.choice([0, 50], n).astype(np.float32)
    ph = rng.uniform(0.1, 4, (n, T)).astype(np.float32)
    ph[::17, 3] = 0.0
    c = kbm.sigmag_coeff(ql, qh)
    keep, lh, ok = kbm.sigmag_filter_ex(_cuda(ps), _cuda(ph), quantity=quantity, q_lo=ql,
                                        q_hi=qh, coeff=c, lh_min=2.0)
    rk, rl = oracle_mod.sigmag(ps, ph, q_lo=ql, q_hi=qh, coeff=c, quantity=quantity)
    assert np.array_equal(keep.cpu().numpy().view(np.uint64), rk)
    assert np.all(P.lh_close(lh.cpu().numpy(), rl))
    g_ok = ok.cpu().numpy()
    near = np.abs(rl - 2.0) <= 1e-4 * np.maximum(np.abs(rl), 1.0)
    assert np.all((g_ok == (rl >= 2.0)) | near)
