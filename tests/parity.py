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
