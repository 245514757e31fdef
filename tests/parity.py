"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (derived, stated once here):
  * Planes: binary32 accumulation of k^2 terms; |delta| <= 1e-5 * sum|terms|
    (the FP32 sum bound gamma_{k^2} * sum|terms| is ~5e-6 for k = 9).
  * Likelihoods (L', L, in sigma units): |delta| <= 1e-4 * max(|L_ref|, 1).
  * Keep masks: bit-identical when both sides read the same float32 planes
    (the decision is taken in binary32 on both sides).
  * Top-K: where the velocity chosen for a slot differs, the oracle's L' of
    both choices must agree to the likelihood tolerance (a near tie);
    everything else must be identical.
"""
import numpy as np

LH_TOL = 1e-4
U32 = 2.0 ** -24   # unit roundoff of binary32


def f32_margin_bound(numax, coeff=0.7413, n_sigma=2.0):
    """Largest amount by which a binary32 evaluation of the sigma_G decision
    margin m = |nu_i - x_50| - n C (x_hi - x_lo) can differ from its exact
    (FP64) value, for a lightcurve whose largest |nu| is ``numax`` (u = 2^-24,
    correctly rounded operations, no contraction):
      * nu = psi / sqrt(phi) carries two roundings: |d nu| <= 2.01 u numax
        (psi/phi: one rounding, less);
      * order statistics are 1-Lipschitz in the max norm, so each selected
        x_q moves by at most 2.01 u numax;
      * x_hi - x_lo: 4.02 u numax from the inputs plus one rounding of a
        value <= 2 numax: <= 6.1 u numax; then the products by C and n
        (binary32 C carries its own rounding) add 3.01 u of <= 2 n C numax:
        the threshold moves by <= 12.2 n C u numax;
      * |nu_i - x_50|: 4.02 u numax from the inputs plus one rounding of a
        value <= 2 numax: <= 6.03 u numax.
    The sum, rounded up: (7 + 14 n C) u numax."""
    return (7.0 + 14.0 * n_sigma * coeff) * U32 * np.asarray(numax, np.float64)


def to_np(out):
    r = {}
    for k, v in out.items():
        if v is None:
            continue
        a = v.detach().cpu().numpy()
        if k == "keep":
            a = a.view(np.uint64)
        r[k] = a
    return r


def lh_close(a, b, tol=LH_TOL):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    both_inf = np.isneginf(a) & np.isneginf(b)
    with np.errstate(invalid="ignore"):
        err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    return both_inf | (err <= tol)


def compare_search(g, r, single_eval=None, tol=LH_TOL, max_tie_frac=0.01):
    """Compare GPU results ``g`` with oracle results ``r`` slot by slot.

    ``single_eval(y, x, v)`` returns the oracle's L' of velocity v at region
    pixel (y, x) (or -inf), used to validate near-tie swaps.  Returns a dict
    of counts; raises AssertionError on any violation."""
    g = to_np(g) if not isinstance(g["lh"], np.ndarray) else g
    assert g["lh"].shape == r["lh"].shape, (g["lh"].shape, r["lh"].shape)
    same = g["vel_idx"] == r["vel_idx"]
    diff = ~same
    n_diff = int(diff.sum())
    # identical choices: every field must agree
    assert np.array_equal(g["n_obs"][same].astype(np.int64), r["n_obs"][same].astype(np.int64))
    bad_keep = int(np.sum(g["keep"][same] != r["keep"][same].astype(np.uint64)))
    assert bad_keep == 0, f"{bad_keep} keep masks differ"
    ok = lh_close(g["lh"][same], r["lh"][same], tol)
    assert ok.all(), _worst(g["lh"][same], r["lh"][same])
    if "lh_raw" in g:
        ok = lh_close(g["lh_raw"][same], r["lh_raw"][same], tol)
        assert ok.all(), _worst(g["lh_raw"][same], r["lh_raw"][same])
    fl_ok = np.abs(g["flux"][same] - r["flux"][same]) <= tol * np.maximum(
        np.abs(r["flux"][same]), 1.0)
    assert fl_ok.all()
    # differing choices: must be near ties under the oracle's likelihood
    if n_diff:
        assert n_diff <= max_tie_frac * same.size + 4, f"{n_diff} slots differ"
        assert single_eval is not None, f"{n_diff} slots differ"
        for (y, x, s) in np.argwhere(diff):
            gv = int(g["vel_idx"][y, x, s])
            ref = float(r["lh"][y, x, s])
            assert gv >= 0 and r["vel_idx"][y, x, s] >= 0, (y, x, s)
            lg = single_eval(int(y), int(x), gv)
            assert lh_close(lg, ref, tol), (y, x, s, gv, lg, ref)
            assert lh_close(g["lh"][y, x, s], ref, tol), (y, x, s)
    return dict(slots=int(same.size), tie_swaps=n_diff)


def _worst(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fin = np.isfinite(a) & np.isfinite(b)
    with np.errstate(invalid="ignore"):
        err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    err[~fin] = np.where(a[~fin] == b[~fin], 0, np.inf)
    i = int(np.argmax(err))
    return f"worst at {i}: gpu={a.flat[i]} ref={b.flat[i]} err={err.flat[i]}"


def plane_terms_abs(oracle_mod, sci, var, mask, psf):
    """sum |terms| of the psi correlation: psi of |I| with |P|."""
    a, _ = oracle_mod.planes(np.abs(sci), var, mask, np.abs(psf))
    return a


def _bits(words, T):
    w = np.asarray(words, np.uint64)
    return ((w[:, None] >> np.arange(T, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(bool)


def certify_fp64(oracle_mod, g, psi, phi, times, vels, p, region=(0, 0)):
    """Certify the GPU's binary32 keep decisions against the FP64 decision.

    Every GPU result slot (vel_idx >= 0) of ``g`` (searched over the float32
    planes ``psi``, ``phi``) is re-evaluated by the oracle with the binary64
    decision; each keep bit where the two differ must have an FP64 margin
    |nu_i - x_50| - thr within ``f32_margin_bound``.  Returns counts (slots,
    differing bits, slots with any, largest |margin| / bound among them)."""
    gn = to_np(g) if not isinstance(g["lh"], np.ndarray) else g
    ys, xs, ss = np.nonzero(gn["vel_idx"] >= 0)
    if ys.size == 0:
        return dict(slots=0, bits_differ=0, slots_differ=0, worst_ratio=0.0)
    starts = np.stack([xs + region[0], ys + region[1]], 1)
    vel = np.asarray(vels, np.float32)[gn["vel_idx"][ys, xs, ss]]
    q = {k: p[k] for k in ("min_obs", "sigmag", "q_lo", "q_hi", "coeff", "n_sigma")}
    ev = oracle_mod.eval_grid(psi, phi, times, starts, vel, decision="f64",
                              want_margin=True, **q)
    assert np.all(np.isfinite(ev["lh"])), "a GPU result is dropped by the FP64 decision"
    T = psi.shape[0]
    diff = _bits(gn["keep"][ys, xs, ss] ^ ev["keep"], T)
    bound = f32_margin_bound(ev["numax"], p["coeff"], p["n_sigma"])[:, None]
    m = np.abs(ev["margin"])
    assert np.all(np.isfinite(m[diff])), "a differing bit on an epoch that does not take part"
    ok = m <= bound
    bad = diff & ~ok
    assert not bad.any(), (f"{int(bad.sum())} keep bits differ from the FP64 decision "
                           f"beyond the binary32 bound; worst margin/bound "
                           f"{float(np.max(m[bad] / np.broadcast_to(bound, m.shape)[bad]))}")
    ratio = (m / np.maximum(bound, 1e-300))[diff]
    return dict(slots=int(ys.size), bits_differ=int(diff.sum()),
                slots_differ=int(diff.any(axis=1).sum()),
                worst_ratio=float(ratio.max()) if ratio.size else 0.0)


def lightcurve(planes, times, vel, x, y, oracle_mod):
    """Values of each plane in ``planes`` along the grid trajectory from
    (x, y) with velocity ``vel``, and the in-image flags (offsets from the
    oracle's offset table)."""
    T, H, W = planes[0].shape
    off = oracle_mod.offsets(times, np.asarray(vel, np.float32).reshape(1, 2))[0]
    xx, yy = x + off[:, 0], y + off[:, 1]
    inside = (xx >= 0) & (xx < W) & (yy >= 0) & (yy < H)
    xc, yc = np.clip(xx, 0, W - 1), np.clip(yy, 0, H - 1)
    t = np.arange(T)
    return [np.where(inside, pl[t, yc, xc], 0.0) for pl in planes], inside


def compare_protocol_c(oracle_mod, g, r, opsi, ophi, terms, times, vels, p,
                       gpu_eval, region=(0, 0), tol=LH_TOL):
    """Protocol C: the GPU searched its own planes, the oracle its planes
    rounded to float32 (``opsi``, ``ophi``); ``terms`` is sum|terms| of the
    psi correlation per pixel-epoch (the protocol-A bound is 1e-5 of it).

    Every GPU slot must be explained by the oracle: at the GPU's chosen
    velocity either the keep mask equals the oracle's and L' agrees to
    ``tol``, or every differing keep bit is certified (its FP64 margin lies
    within the plane-error bound plus both sides' binary32 bound) and the
    GPU's L' equals, to ``tol``, the oracle-plane L' over the GPU's keep
    mask.  Where the chosen velocities differ, the two choices must be a
    near tie (to ``tol``) or one of them must carry a certified keep flip
    (``gpu_eval(x, y, v)`` gives the GPU's (keep, L') of any trajectory).
    Returns counts."""
    gn = to_np(g) if not isinstance(g["lh"], np.ndarray) else g
    T = opsi.shape[0]
    q = {k: p[k] for k in ("min_obs", "sigmag", "q_lo", "q_hi", "coeff", "n_sigma")}
    nc = p["n_sigma"] * p["coeff"]
    vels = np.asarray(vels, np.float32)
    stats = dict(slots=0, flips_certified=0, flip_bits=0, vel_swaps=0,
                 swaps_near_tie=0, swaps_by_flip=0)

    def certify_flip(x, y, v, keep_g, lh_g, k_o):
        """The GPU keep mask of (x, y, v) differs from the oracle's k_o:
        certify every differing bit and the GPU's L' over its own mask."""
        ev = oracle_mod.eval_grid(opsi, ophi, times, [[x, y]], vels[v:v + 1],
                                  decision="f64", want_margin=True, **q)
        (ps, ph, tm), inside = lightcurve([opsi, ophi, terms], times, vels[v], x, y,
                                          oracle_mod)
        ps, ph, tm = (a.astype(np.float64) for a in (ps, ph, tm))
        part = inside & (ph > 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            nu = np.where(part, ps / np.sqrt(ph), 0.0)
            dnu = np.where(part, 1.01e-5 * tm / np.sqrt(ph) + 0.6e-5 * np.abs(nu), 0.0)
        bound = ((2.0 + 2.0 * nc) * dnu.max()
                 + 2.0 * f32_margin_bound(ev["numax"][0], p["coeff"], p["n_sigma"]))
        flip = _bits(np.array([keep_g ^ k_o], np.uint64), T)[0]
        m = ev["margin"][0]
        assert np.all(np.isfinite(m[flip])), (x, y, v)
        assert np.all(np.abs(m[flip]) <= bound), (x, y, v, m[flip], bound)
        kb = _bits(np.array([keep_g], np.uint64), T)[0]
        sp, sf = ps[kb].sum(), ph[kb].sum()
        assert lh_close(lh_g, sp / np.sqrt(sf), tol), (x, y, v, lh_g, sp / np.sqrt(sf))
        stats["flips_certified"] += 1
        stats["flip_bits"] += int(flip.sum())

    ys, xs, ss = np.nonzero(gn["vel_idx"] >= 0)
    X, Y = xs + region[0], ys + region[1]
    vg = gn["vel_idx"][ys, xs, ss]
    stats["slots"] = int(ys.size)
    e32 = oracle_mod.eval_grid(opsi, ophi, times, np.stack([X, Y], 1), vels[vg], **q)
    kg = gn["keep"][ys, xs, ss]
    lg = gn["lh"][ys, xs, ss]
    same_keep = kg == e32["keep"]
    ok = lh_close(lg[same_keep], e32["lh"][same_keep], tol)
    assert ok.all(), _worst(lg[same_keep], e32["lh"][same_keep])
    assert np.array_equal(gn["n_obs"][ys, xs, ss].astype(np.int64),
                          e32["n_obs"].astype(np.int64))
    flip_g = ~same_keep
    for j in np.nonzero(flip_g)[0]:
        certify_flip(int(X[j]), int(Y[j]), int(vg[j]), int(kg[j]), float(lg[j]),
                     int(e32["keep"][j]))
    vo = r["vel_idx"][ys, xs, ss]
    for j in np.nonzero(vg != vo)[0]:
        stats["vel_swaps"] += 1
        assert vo[j] >= 0, "GPU fills a slot the oracle leaves empty"
        lo = float(r["lh"][ys[j], xs[j], ss[j]])
        if lh_close(lg[j], lo, tol):
            stats["swaps_near_tie"] += 1
            continue
        x, y, v = int(X[j]), int(Y[j]), int(vo[j])
        kg_o, lg_o = gpu_eval(x, y, v)
        k_o = int(r["keep"][ys[j], xs[j], ss[j]])
        flip_o = kg_o != k_o
        if flip_o:
            certify_flip(x, y, v, kg_o, lg_o, k_o)
        assert flip_g[j] or flip_o, (x, y, int(vg[j]), v, float(lg[j]), lo)
        stats["swaps_by_flip"] += 1
    # slots the oracle fills must be filled on the GPU too
    assert np.array_equal(gn["vel_idx"] >= 0, r["vel_idx"] >= 0)
    return stats
