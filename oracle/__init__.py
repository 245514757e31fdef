"""Plain FP64 CPU oracle for the shift-and-stack search (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import it; the two share no code, only the seeded input arrays from
``synth``.

The arithmetic lives in ``kbm_oracle.c`` (plain C loops transcribing the
definitions; see that file's header for the passages each function
follows).  This module builds it with gcc and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kbm_oracle.c")
_LIB = os.path.join(_HERE, "libkbm_oracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-std=c99"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        lib.kbmo_planes.argtypes = [i32, i32, i32, P, P, P, P, i32, P, P]
        lib.kbmo_offsets.argtypes = [i32, P, i32, P, P]
        lib.kbmo_offsets.restype = None
        lib.kbmo_sigmag.argtypes = [i64, i32, P, P, P, f64, f64, f64, f64, P, P]
        lib.kbmo_sigmag_q.argtypes = [i64, i32, P, P, P, i32, f64, f64, f64, f64,
                                      P, P]
        lib.kbmo_search.argtypes = [i32, i32, i32, P, P, P, i32, P, i32, i32,
                                    i32, f64, f64, f64, f64, i32, i32, i32,
                                    i32, P, P, P, P, P, P]
        lib.kbmo_search_ex.argtypes = [i32, i32, i32, P, P, P, i32, P, i32, i32,
                                       i32, i32, f64, f64, f64, f64, i32, i32, i32,
                                       i32, P, P, P, P, P, P]
        lib.kbmo_sigmag_ex.argtypes = [i64, i32, P, P, P, i32, i32, f64, f64, f64,
                                       f64, P, P, P, P]
        lib.kbmo_eval_grid.argtypes = [i32, i32, i32, P, P, P, i64, P, P, i32, i32,
                                       i32, f64, f64, f64, f64, P, P, P, P, P, P, P]
        lib.kbmo_refine.argtypes = [i32, i32, i32, P, P, P, i64, P, P, P, P,
                                    P, P, P]
        lib.kbmo_score.argtypes = [i32, i32, i32, P, P, P, i64, P, i32, i32, f64,
                                   f64, f64, f64, P, P, P, P, P]
        lib.kbmo_num_threads.restype = C.c_int
        lib.kbmo_set_num_threads.argtypes = [C.c_int]
        lib.kbmo_set_num_threads.restype = None
        _lib = lib
        return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(_load().kbmo_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on (OpenMP)."""
    _load().kbmo_set_num_threads(int(n))


def planes(sci, var, mask, psf):
    """FP64 psi/phi planes ``[T][H][W]`` (PSF correlation, masked = weight 0)."""
    lib = _load()
    sci, var = _c(sci, np.float32), _c(var, np.float32)
    mask = _c(mask, np.uint8)
    psf = _c(psf, np.float32)
    T, H, W = sci.shape
    k = psf.shape[0]
    psi = np.empty((T, H, W), np.float64)
    phi = np.empty((T, H, W), np.float64)
    rc = lib.kbmo_planes(T, H, W, _p(sci), _p(var), _p(mask), _p(psf), k,
                         _p(psi), _p(phi))
    if rc:
        raise ValueError("oracle planes: bad arguments")
    return psi, phi


def offsets(times, vels):
    """int32 ``[V][T][2]`` offsets floor(v*t + 1/2), t from the earliest epoch."""
    lib = _load()
    times = _c(times, np.float64)
    vels = _c(vels, np.float32).reshape(-1, 2)
    T, V = times.shape[0], vels.shape[0]
    off = np.empty((V, T, 2), np.int32)
    lib.kbmo_offsets(T, _p(times), V, _p(vels), _p(off))
    return off


DECISIONS = {"f32": 0, "f64": 1}


def _decision(d):
    if d not in DECISIONS:
        raise ValueError(f"decision must be one of {sorted(DECISIONS)}")
    return DECISIONS[d]


def sigmag(psi_curve, phi_curve=None, valid=None, q_lo=0.25, q_hi=0.75,
           coeff=0.7413, n_sigma=2.0, quantity=0, decision="f32",
           want_margin=False):
    """Standalone sigma_G filter over ``[n][T]`` lightcurves (Section 3.1);
    ``quantity`` 0 filters psi/sqrt(phi) (likelihood), 1 psi/phi (flux).
    ``decision`` is the precision of the keep decision ("f32": binary32,
    "f64": binary64).

    Returns (keep uint64 [n], lh float64 [n]), plus, with ``want_margin``,
    the FP64 margins |nu_i - x_50| - thr ``[n][T]`` (NaN where an epoch does
    not take part) and the largest |nu_i| per lightcurve ``[n]``."""
    lib = _load()
    ps = _c(psi_curve, np.float32)
    n, T = ps.shape
    ph = _c(phi_curve, np.float32)
    va = _c(valid, np.uint8)
    keep = np.empty(n, np.uint64)
    lh = np.empty(n, np.float64)
    margin = np.empty((n, T), np.float64) if want_margin else None
    numax = np.empty(n, np.float64) if want_margin else None
    rc = lib.kbmo_sigmag_ex(n, T, _p(ps), _p(ph), _p(va), int(quantity),
                            _decision(decision), q_lo, q_hi, coeff, n_sigma,
                            _p(keep), _p(lh), _p(margin), _p(numax))
    if rc:
        raise ValueError("oracle sigmag: bad arguments")
    if want_margin:
        return keep, lh, margin, numax
    return keep, lh


def search(psi, phi, times, vels, *, k=8, min_obs=1, sigmag=1, q_lo=0.25,
           q_hi=0.75, coeff=0.7413, n_sigma=2.0, region=None, decision="f32",
           **_ignored):
    """Exhaustive search over float32 planes.

    ``region = (x_begin, y_begin, x_end, y_end)`` (default: whole image);
    ``decision`` the precision of the sigma_G keep decision ("f32", "f64").
    Returns a dict of ``[Hr][Wr][k]`` arrays: lh (filtered likelihood),
    flux, vel_idx, n_obs, keep, lh_raw."""
    lib = _load()
    psi, phi = _c(psi, np.float32), _c(phi, np.float32)
    times = _c(times, np.float64)
    vels = _c(vels, np.float32).reshape(-1, 2)
    T, H, W = psi.shape
    if region is None:
        region = (0, 0, W, H)
    x0, y0, x1, y1 = (int(v) for v in region)
    Hr, Wr = y1 - y0, x1 - x0
    out = dict(lh=np.empty((Hr, Wr, k), np.float64),
               flux=np.empty((Hr, Wr, k), np.float64),
               vel_idx=np.empty((Hr, Wr, k), np.int32),
               n_obs=np.empty((Hr, Wr, k), np.int32),
               keep=np.empty((Hr, Wr, k), np.uint64),
               lh_raw=np.empty((Hr, Wr, k), np.float64))
    rc = lib.kbmo_search_ex(T, H, W, _p(psi), _p(phi), _p(times), vels.shape[0],
                            _p(vels), k, min_obs, int(sigmag), _decision(decision),
                            q_lo, q_hi, coeff, n_sigma, x0, y0, x1, y1, _p(out["lh"]),
                            _p(out["flux"]), _p(out["vel_idx"]), _p(out["n_obs"]),
                            _p(out["keep"]), _p(out["lh_raw"]))
    if rc:
        raise ValueError("oracle search: bad arguments (rc=%d)" % rc)
    return out


def eval_grid(psi, phi, times, starts, vels, *, min_obs=1, sigmag=1, q_lo=0.25,
              q_hi=0.75, coeff=0.7413, n_sigma=2.0, decision="f32",
              want_margin=False, **_ignored):
    """Evaluate explicit grid trajectories exactly as the search does:
    ``starts`` int ``[n][2]`` start pixels (x, y), ``vels`` ``[n][2]``
    velocities (px/day).  Returns a dict of ``[n]`` arrays lh, flux, keep,
    n_obs, lh_raw (lh = -inf where the search would drop the trajectory),
    and with ``want_margin`` the FP64 decision margins ``margin`` [n][T]
    and ``numax`` [n] (see ``sigmag``)."""
    lib = _load()
    psi, phi = _c(psi, np.float32), _c(phi, np.float32)
    times = _c(times, np.float64)
    starts = _c(starts, np.int32).reshape(-1, 2)
    vels = _c(vels, np.float32).reshape(-1, 2)
    T, H, W = psi.shape
    n = starts.shape[0]
    if vels.shape[0] != n:
        raise ValueError("eval_grid: starts and vels differ in length")
    out = dict(lh=np.empty(n, np.float64), flux=np.empty(n, np.float64),
               keep=np.empty(n, np.uint64), n_obs=np.empty(n, np.int32),
               lh_raw=np.empty(n, np.float64))
    if want_margin:
        out["margin"] = np.empty((n, T), np.float64)
        out["numax"] = np.empty(n, np.float64)
    rc = lib.kbmo_eval_grid(T, H, W, _p(psi), _p(phi), _p(times), n, _p(starts),
                            _p(vels), int(min_obs), int(sigmag), _decision(decision),
                            q_lo, q_hi, coeff, n_sigma, _p(out["lh"]), _p(out["flux"]),
                            _p(out["keep"]), _p(out["n_obs"]), _p(out["lh_raw"]),
                            _p(out.get("margin")), _p(out.get("numax")))
    if rc:
        raise ValueError("oracle eval_grid: bad arguments")
    return out


def refine(psi, phi, times, params, keep=None, grad_lh=None, want_planes=False):
    """Bilinear refinement objective L for ``[n][4]`` params (x0, y0, vx, vy).

    With ``grad_lh`` given, also returns g * dL/dparams and, if
    ``want_planes``, the accumulated dL/dpsi and dL/dphi planes."""
    lib = _load()
    psi, phi = _c(psi, np.float32), _c(phi, np.float32)
    times = _c(times, np.float64)
    params = _c(params, np.float32).reshape(-1, 4)
    T, H, W = psi.shape
    n = params.shape[0]
    keep = _c(keep, np.uint64)
    g = _c(grad_lh, np.float64)
    lh = np.empty(n, np.float64)
    gp = np.zeros((n, 4), np.float64) if g is not None else None
    gpsi = np.zeros((T, H, W), np.float64) if (g is not None and want_planes) else None
    gphi = np.zeros((T, H, W), np.float64) if (g is not None and want_planes) else None
    rc = lib.kbmo_refine(T, H, W, _p(psi), _p(phi), _p(times), n, _p(params),
                         _p(keep), _p(g), _p(lh), _p(gp), _p(gpsi), _p(gphi))
    if rc:
        raise ValueError("oracle refine: bad arguments")
    if g is None:
        return lh
    if want_planes:
        return lh, gp, gpsi, gphi
    return lh, gp


def score(psi, phi, times, params, *, min_obs=1, sigmag=1, q_lo=0.25,
          q_hi=0.75, coeff=0.7413, n_sigma=2.0, **_ignored):
    """Targeted evaluation of ``[n][4]`` float32 trajectories (x0, y0, vx,
    vy) with real-valued starts: the search's L' at the pixels
    floor(x0 + vx t + 1/2), floor(y0 + vy t + 1/2).  Returns a dict of
    ``[n]`` arrays lh, flux, keep, n_obs, lh_raw."""
    lib = _load()
    psi, phi = _c(psi, np.float32), _c(phi, np.float32)
    times = _c(times, np.float64)
    params = _c(params, np.float32).reshape(-1, 4)
    T, H, W = psi.shape
    n = params.shape[0]
    out = dict(lh=np.empty(n, np.float64), flux=np.empty(n, np.float64),
               keep=np.empty(n, np.uint64), n_obs=np.empty(n, np.int32),
               lh_raw=np.empty(n, np.float64))
    rc = lib.kbmo_score(T, H, W, _p(psi), _p(phi), _p(times), n, _p(params),
                        int(min_obs), int(sigmag), q_lo, q_hi, coeff, n_sigma,
                        _p(out["lh"]), _p(out["flux"]), _p(out["keep"]),
                        _p(out["n_obs"]), _p(out["lh_raw"]))
    if rc:
        raise ValueError("oracle score: bad arguments")
    return out


def extract_top(lh, n_max, lh_min=-np.inf):
    """Global top-N slots of a search result ``lh`` [Hr][Wr][K] (plain
    definition): qualifying slots are finite with L' >= lh_min; rank by L'
    descending then flat slot index ascending; keep the first n_max; return
    their flat indices in increasing order."""
    flat = np.asarray(lh, np.float64).ravel()
    idx = np.arange(flat.size)
    ok = np.isfinite(flat) & (flat >= lh_min)
    order = np.lexsort((idx[ok], -flat[ok]))
    return np.sort(idx[ok][order][:n_max])


def adam_step(p, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8,
              maximize=True):
    """One Adam update (Kingma & Ba, Algorithm 1) in FP64, per-column lr.
    Returns new (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    g = -g if maximize else g
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p = p - np.asarray(lr, np.float64) * mh / (np.sqrt(vh) + eps)
    return p, m, v


STAMP_LIMITS = (0.5, 0.5, 1.5, 36.5, 36.5)   # |x|, |y|, |xy|, xx, yy (Section 3.3)


def sigmag_coeff(q_lo, q_hi):
    """C of Eq. 3 for a quantile pair: 1 / (sqrt(2) (erfinv(2 q_hi - 1) -
    erfinv(2 q_lo - 1))), so that C (x_hi - x_lo) estimates sigma for normal
    data (0.7413 for the 25th/75th percentiles, Section 3.1)."""
    from scipy.special import erfinv
    return 1.0 / (math.sqrt(2.0) * (erfinv(2.0 * q_hi - 1.0) - erfinv(2.0 * q_lo - 1.0)))


def stamps(sci, var, mask, times, params, radius=10, keep=None):
    """Median coadded postage stamps along trajectories (Section 3.3):
    for each trajectory (params [n][4] = x0, y0, vx, vy, float32) and epoch
    i, the (2r+1)^2 window of the science image centred on the pixel
    (floor(x0 + vx t_i + 1/2), floor(y0 + vy t_i + 1/2)); a pixel of an epoch
    is usable when it lies in the image, is unmasked, and sci, var are
    finite with var > 0 (and, with ``keep`` given, the epoch's keep bit is
    set).  The coadd is numpy's median of the usable values of each stamp
    pixel (mean of the two middle values for an even count), 0 where none is
    usable.  Returns float32 [n][2r+1][2r+1]."""
    sci = np.asarray(sci, np.float32)
    var = np.asarray(var, np.float32)
    T, H, W = sci.shape
    times = np.asarray(times, np.float64)
    t = times - times.min()
    params = np.asarray(params, np.float32).reshape(-1, 4)
    n = params.shape[0]
    k = 2 * radius + 1
    ok_pix = np.isfinite(sci) & np.isfinite(var) & (var > 0)
    if mask is not None:
        ok_pix &= np.asarray(mask) == 0
    out = np.zeros((n, k, k), np.float32)
    d = np.arange(-radius, radius + 1)
    for j in range(n):
        x0, y0, vx, vy = (float(v) for v in params[j])
        cube = np.full((T, k, k), np.nan, np.float32)
        for i in range(T):
            if keep is not None and not (int(keep[j]) >> i) & 1:
                continue
            cx = math.floor(x0 + vx * t[i] + 0.5)
            cy = math.floor(y0 + vy * t[i] + 0.5)
            ys, xs = cy + d, cx + d
            iny = (ys >= 0) & (ys < H)
            inx = (xs >= 0) & (xs < W)
            sub = np.full((k, k), np.nan, np.float32)
            yy, xx = np.ix_(np.where(iny)[0], np.where(inx)[0])
            src_y, src_x = np.ix_(ys[iny], xs[inx])
            vals = sci[i][src_y, src_x]
            good = ok_pix[i][src_y, src_x]
            sub[yy, xx] = np.where(good, vals, np.nan)
            cube[i] = sub
        with np.errstate(all="ignore"):
            import warnings
            with warnings.catch_warnings():
                warnings.simplefilter("ignore", RuntimeWarning)
                med = np.nanmedian(cube, axis=0)
        out[j] = np.where(np.isnan(med), np.float32(0), med).astype(np.float32)
    return out


def stamp_moments(stamp):
    """Central moments of a coadded stamp (Section 3.3) in FP64: with
    S normalised to unit sum and offsets dx, dy from the centre pixel,
    (sum, x, y, xy, xx, yy) = (sum S, sum dx S, sum dy S, sum dx dy S,
    sum dx^2 S, sum dy^2 S).  A stamp whose sum is not positive gets NaN
    moments."""
    s = np.asarray(stamp, np.float64)
    k = s.shape[-1]
    r = k // 2
    d = np.arange(-r, r + 1, dtype=np.float64)
    tot = s.sum(axis=(-1, -2))
    with np.errstate(all="ignore"):
        w = s / tot[..., None, None]
    dx = d[None, :]
    dy = d[:, None]
    m = np.stack([tot, (w * dx).sum((-1, -2)), (w * dy).sum((-1, -2)),
                  (w * dx * dy).sum((-1, -2)), (w * dx * dx).sum((-1, -2)),
                  (w * dy * dy).sum((-1, -2))], -1)
    m[..., 1:] = np.where((tot > 0)[..., None], m[..., 1:], np.nan)
    return m


def stamp_pass(moments, limits=STAMP_LIMITS):
    """The central-moment cut of Section 3.3: |x|, |y|, |xy| and xx, yy all
    strictly below their limits (NaN moments fail)."""
    m = np.asarray(moments, np.float64)
    lx, ly, lxy, lxx, lyy = limits
    with np.errstate(invalid="ignore"):
        return ((np.abs(m[..., 1]) < lx) & (np.abs(m[..., 2]) < ly) &
                (np.abs(m[..., 3]) < lxy) & (m[..., 4] < lxx) & (m[..., 5] < lyy))
