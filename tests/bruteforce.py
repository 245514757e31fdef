"""Independent brute-force evaluations for tiny inputs.

Written straight from the definitions with different machinery from the C
oracle: planes through ``scipy.ndimage.correlate``, trajectory sums with
``math.fsum``, order statistics with Python's ``sorted``, the per-pixel top-K
by sorting *every* candidate of a pixel, and bilinear samples through
``scipy.ndimage.map_coordinates``.  Used only on inputs small enough for
pure-Python loops.
"""
import math

import numpy as np
from scipy import ndimage

F32 = np.float32


def weights(sci, var, mask):
    """Inverse variance where the pixel is usable, zero elsewhere."""
    ok = np.isfinite(sci) & np.isfinite(var) & (var > 0)
    if mask is not None:
        ok &= (mask == 0)
    w = np.zeros(sci.shape, np.float64)
    w[ok] = 1.0 / var[ok].astype(np.float64)
    iw = np.zeros(sci.shape, np.float64)
    iw[ok] = sci[ok].astype(np.float64) * w[ok]
    return w, iw


def planes(sci, var, mask, psf):
    """psi = corr(I*w, P), phi = corr(w, P^2), zero outside the image."""
    w, iw = weights(sci, var, mask)
    p = psf.astype(np.float64)
    psi = np.stack([ndimage.correlate(iw[t], p, mode="constant", cval=0.0)
                    for t in range(sci.shape[0])])
    phi = np.stack([ndimage.correlate(w[t], p * p, mode="constant", cval=0.0)
                    for t in range(sci.shape[0])])
    return psi, phi


def offset(v, t):
    return int(math.floor(float(v) * float(t) + 0.5))


def sigmag_keep(values_psi, values_phi, q_lo, q_hi, coeff, n_sigma):
    """Keep flags for a list of (psi, phi) samples, binary32 decisions."""
    nu = [F32(a) / np.sqrt(F32(b)) for a, b in zip(values_psi, values_phi)]
    n = len(nu)
    if n == 0:
        return []
    s = sorted(nu)

    def q(qq):
        return s[int(math.floor(qq * (n - 1) + 0.5))]

    x_lo, x_md, x_hi = q(q_lo), q(0.5), q(q_hi)
    sig = F32(coeff) * F32(x_hi - x_lo)
    thr = F32(n_sigma) * sig
    return [bool(abs(F32(x - x_md)) <= thr) for x in nu]


def sigmag_keep64(values_psi, values_phi, q_lo, q_hi, coeff, n_sigma):
    """Keep flags for a list of (psi, phi) samples, the decision taken in
    Python floats (binary64) straight from Eqs. 1-5: nu = psi/sqrt(phi),
    nearest-rank quantiles of the sorted values, sigma_G = C (x_hi - x_lo),
    keep when |nu - x_50| <= n sigma_G."""
    nu = [float(a) / math.sqrt(float(b)) for a, b in zip(values_psi, values_phi)]
    n = len(nu)
    if n == 0:
        return []
    s = sorted(nu)

    def q(qq):
        return s[int(math.floor(qq * (n - 1) + 0.5))]

    thr = n_sigma * (coeff * (q(q_hi) - q(q_lo)))
    return [abs(x - q(0.5)) <= thr for x in nu]


def trajectory(psi, phi, times, vel, x, y, sigmag, q_lo, q_hi, coeff, n_sigma,
               decision="f32"):
    """Evaluate one trajectory; returns None when it has no usable epoch."""
    T, H, W = psi.shape
    t0 = min(times)
    idx, ps, ph = [], [], []
    for i in range(T):
        xx = x + offset(vel[0], times[i] - t0)
        yy = y + offset(vel[1], times[i] - t0)
        if not (0 <= xx < W and 0 <= yy < H):
            continue
        a, b = psi[i, yy, xx], phi[i, yy, xx]
        if not (b > 0 and np.isfinite(a) and np.isfinite(b)):
            continue
        idx.append(i)
        ps.append(float(a))
        ph.append(float(b))
    if not idx:
        return None
    lraw = math.fsum(ps) / math.sqrt(math.fsum(ph))
    if sigmag:
        rule = sigmag_keep64 if decision == "f64" else sigmag_keep
        kf = rule(ps, ph, q_lo, q_hi, coeff, n_sigma)
    else:
        kf = [True] * len(idx)
    kp = [a for a, k in zip(ps, kf) if k]
    kh = [b for b, k in zip(ph, kf) if k]
    keep = 0
    for i, k in zip(idx, kf):
        if k:
            keep |= 1 << i
    sp, sf = math.fsum(kp), math.fsum(kh)
    return dict(lh=sp / math.sqrt(sf), flux=sp / sf, n_obs=len(idx),
                keep=keep, lh_raw=lraw)


def trajectory_real(psi, phi, times, prm, sigmag, q_lo, q_hi, coeff, n_sigma):
    """One trajectory with a real-valued start: epoch i samples pixel
    floor(x0 + vx t_i + 1/2) (Python floats, evaluated left to right)."""
    T, H, W = psi.shape
    x0, y0, vx, vy = (float(np.float32(v)) for v in prm)
    t0 = min(times)
    idx, ps, ph = [], [], []
    for i in range(T):
        t = float(times[i]) - float(t0)
        xx = math.floor(x0 + vx * t + 0.5)
        yy = math.floor(y0 + vy * t + 0.5)
        if not (0 <= xx < W and 0 <= yy < H):
            continue
        a, b = psi[i, yy, xx], phi[i, yy, xx]
        if not (b > 0 and np.isfinite(a) and np.isfinite(b)):
            continue
        idx.append(i)
        ps.append(float(a))
        ph.append(float(b))
    if not idx:
        return None
    lraw = math.fsum(ps) / math.sqrt(math.fsum(ph))
    kf = (sigmag_keep(ps, ph, q_lo, q_hi, coeff, n_sigma) if sigmag
          else [True] * len(idx))
    kp = [a for a, k in zip(ps, kf) if k]
    kh = [b for b, k in zip(ph, kf) if k]
    keep = 0
    for i, k in zip(idx, kf):
        if k:
            keep |= 1 << i
    sp, sf = math.fsum(kp), math.fsum(kh)
    return dict(lh=sp / math.sqrt(sf), flux=sp / sf, n_obs=len(idx),
                keep=keep, lh_raw=lraw)


def search(psi, phi, times, vels, k, min_obs, sigmag=1, q_lo=0.25, q_hi=0.75,
           coeff=0.7413, n_sigma=2.0, region=None, decision="f32"):
    T, H, W = psi.shape
    x0, y0, x1, y1 = region or (0, 0, W, H)
    out = dict(lh=np.full((y1 - y0, x1 - x0, k), -np.inf),
               flux=np.zeros((y1 - y0, x1 - x0, k)),
               vel_idx=np.full((y1 - y0, x1 - x0, k), -1, np.int64),
               n_obs=np.zeros((y1 - y0, x1 - x0, k), np.int64),
               keep=np.zeros((y1 - y0, x1 - x0, k), np.uint64),
               lh_raw=np.full((y1 - y0, x1 - x0, k), -np.inf))
    for y in range(y0, y1):
        for x in range(x0, x1):
            cands = []
            for v in range(len(vels)):
                r = trajectory(psi, phi, times, vels[v], x, y, sigmag, q_lo,
                               q_hi, coeff, n_sigma, decision)
                if r is None or r["n_obs"] < min_obs or not math.isfinite(r["lh"]):
                    continue
                cands.append((-r["lh"], v, r))
            cands.sort(key=lambda c: (c[0], c[1]))
            for s, (_, v, r) in enumerate(cands[:k]):
                o = (y - y0, x - x0, s)
                out["lh"][o] = r["lh"]
                out["flux"][o] = r["flux"]
                out["vel_idx"][o] = v
                out["n_obs"][o] = r["n_obs"]
                out["keep"][o] = r["keep"]
                out["lh_raw"][o] = r["lh_raw"]
    return out


def bilinear(plane, x, y):
    """Bilinear sample, pixel centres at integer coordinates, zero outside."""
    return float(ndimage.map_coordinates(plane.astype(np.float64), [[y], [x]],
                                         order=1, mode="grid-constant",
                                         cval=0.0)[0])
