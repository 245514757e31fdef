"""Seeded synthetic difference-image stacks shaped like the paper's DECam data.

This module only *draws inputs*: science, variance and mask planes, the PSF
array, the epoch times and the velocity grid.  It contains none of the search
method's arithmetic (no likelihood planes, no trajectory sums, no filtering);
both the GPU library and the CPU oracle consume exactly the arrays it returns.

Shapes follow the paper's data description (Section 2.1: 2K x 4K DECam CCDs,
about five pointings per night taken roughly five minutes apart, several
nights per pointing group) and the search grid of Section 4.1 (a speed range
times an angle range around the ecliptic).

Recipe (the draw order is part of the contract, so a seed fixes every array):

* ``rng = numpy.random.Generator(numpy.random.PCG64(seed))``.
* Sources are drawn first, one at a time: SNR, speed, angle, then the start
  position (uniform over the box that keeps the whole track at least r+1
  pixels inside the image, r = PSF half-width).
* Then, per epoch in time order: the noise plane N(0,1) (float32), then, if
  the mask rate is non-zero, a uniform plane whose values below the rate mark
  masked pixels.
* A source at epoch e sits at (x0 + vx*t_e, y0 + vy*t_e); its stamp is the
  Gaussian PSF evaluated at integer pixel centres relative to that sub-pixel
  position over a (2r+1)^2 window, scaled to sum to the source flux.
* Difference images are sky subtracted: I = S + sqrt(var) * N(0,1) with
  var = sky + S (Poisson-like).  The tiny configuration instead uses var = 1
  and I = S + N(0,1).
* Flux from the matched-filter per-epoch SNR: f = SNR * sqrt(sky / sum(P^2)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Stack", "psf_size", "gaussian_psf", "night_times", "velocity_grid",
    "make_stack", "make_config", "make_batched_specs", "make_batched_stack",
    "tiny_stack", "default_min_obs", "CONFIG_SEED_BASE",
]

CONFIG_SEED_BASE = 1000
SKY = 100.0
INTRANIGHT_MIN = 5.0      # minutes between exposures within a night
NIGHT_GAP_DAYS = 1.0      # nights are one day apart


@dataclasses.dataclass
class Stack:
    """One aligned stack of difference images plus its search inputs."""
    sci: np.ndarray            # float32 [T][H][W]
    var: np.ndarray            # float32 [T][H][W]
    mask: Optional[np.ndarray]  # uint8 [T][H][W] (nonzero = masked) or None
    psf: np.ndarray            # float32 [k][k]
    times: np.ndarray          # float64 [T] days
    vels: np.ndarray           # float32 [V][2] (vx, vy) px/day
    sources: List[dict]        # injected truth: x0, y0, vx, vy, flux, snr
    params: dict               # search parameters for this configuration
    name: str = ""

    @property
    def T(self) -> int:
        return int(self.sci.shape[0])

    @property
    def H(self) -> int:
        return int(self.sci.shape[1])

    @property
    def W(self) -> int:
        return int(self.sci.shape[2])


def psf_size(sigma: float) -> int:
    """Odd kernel width 2*round(3 sigma)+1 (7, 9, 11 for sigma 1.0, 1.4, 1.6)."""
    return 2 * int(math.floor(3.0 * sigma + 0.5)) + 1


def gaussian_psf(sigma: float, k: Optional[int] = None) -> np.ndarray:
    """Gaussian sampled at pixel centres, normalised to unit sum in float64,
    then stored as float32 ``[k][k]`` (row index = y, column index = x)."""
    if k is None:
        k = psf_size(sigma)
    r = k // 2
    a = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(a[None, :] ** 2 + a[:, None] ** 2) / (2.0 * sigma * sigma))
    g /= g.sum()
    return g.astype(np.float32)


def night_times(n_epochs: int, n_nights: int,
                spacing_min: float = INTRANIGHT_MIN,
                night_gap: float = NIGHT_GAP_DAYS) -> np.ndarray:
    """Epoch times in days since the first epoch.

    Epochs are dealt round-robin to nights (26 over 3 nights gives 9/9/8);
    within a night they are ``spacing_min`` minutes apart."""
    counts = [0] * n_nights
    for e in range(n_epochs):
        counts[e % n_nights] += 1
    t = []
    for n, c in enumerate(counts):
        for j in range(c):
            t.append(n * night_gap + j * spacing_min / 1440.0)
    t = np.sort(np.asarray(t, dtype=np.float64))
    return t - t[0]


def velocity_grid(speeds: Sequence[float], angles: Sequence[float]) -> np.ndarray:
    """Angle-major grid: index = a * len(speeds) + s, (vx, vy) =
    (s cos a, s sin a) evaluated in float64 and stored as float32."""
    sp = np.asarray(speeds, dtype=np.float64)
    an = np.asarray(angles, dtype=np.float64)
    vx = np.cos(an)[:, None] * sp[None, :]
    vy = np.sin(an)[:, None] * sp[None, :]
    return np.stack([vx.ravel(), vy.ravel()], axis=1).astype(np.float32)


def default_min_obs(T: int) -> int:
    """ceil(0.75 T): the paper asks for about 15 observations out of ~20."""
    return int(math.ceil(0.75 * T))


def _stamp(psf_sigma: float, r: int, x: float, y: float, flux: float):
    """Pixel-centred Gaussian around a sub-pixel position, summing to flux."""
    cx = int(math.floor(x + 0.5))
    cy = int(math.floor(y + 0.5))
    xs = np.arange(cx - r, cx + r + 1, dtype=np.float64)
    ys = np.arange(cy - r, cy + r + 1, dtype=np.float64)
    g = np.exp(-((xs[None, :] - x) ** 2 + (ys[:, None] - y) ** 2)
               / (2.0 * psf_sigma * psf_sigma))
    g *= flux / g.sum()
    return cx - r, cy - r, g


def _draw_sources(rng, n, W, H, r, t_max, snr_range, speed_range, angle_range,
                  s2, sky):
    out = []
    for _ in range(n):
        snr = float(rng.uniform(*snr_range))
        speed = float(rng.uniform(*speed_range))
        ang = float(rng.uniform(*angle_range))
        vx, vy = speed * math.cos(ang), speed * math.sin(ang)
        m = r + 1
        dx, dy = vx * t_max, vy * t_max
        xlo, xhi = m - min(0.0, dx), (W - 1 - m) - max(0.0, dx)
        ylo, yhi = m - min(0.0, dy), (H - 1 - m) - max(0.0, dy)
        if xhi <= xlo or yhi <= ylo:
            raise ValueError("image too small for the requested source speeds")
        x0 = float(rng.uniform(xlo, xhi))
        y0 = float(rng.uniform(ylo, yhi))
        flux = snr * math.sqrt(sky / s2)
        out.append(dict(x0=x0, y0=y0, vx=vx, vy=vy, flux=flux, snr=snr))
    return out


def make_stack(W: int, H: int, times: np.ndarray, psf_sigma: float, *,
               seed: int, n_sources: int = 0, snr_range=(3.0, 15.0),
               speed_range=(90.0, 500.0),
               angle_range=(-math.pi / 6, math.pi / 6),
               mask_rate: float = 0.0, sky: float = SKY,
               unit_variance: bool = False, sources: Optional[List[dict]] = None,
               vels: Optional[np.ndarray] = None, params: Optional[dict] = None,
               name: str = "") -> Stack:
    """Draw one stack.  ``sources`` overrides the random source draw."""
    rng = np.random.Generator(np.random.PCG64(seed))
    times = np.asarray(times, dtype=np.float64)
    T = times.shape[0]
    psf = gaussian_psf(psf_sigma)
    k = psf.shape[0]
    r = k // 2
    s2 = float(np.sum(psf.astype(np.float64) ** 2))
    if sources is None:
        sources = _draw_sources(rng, n_sources, W, H, r, float(times.max()),
                                snr_range, speed_range, angle_range, s2, sky)
    sci = np.empty((T, H, W), dtype=np.float32)
    var = np.empty((T, H, W), dtype=np.float32)
    mask = np.zeros((T, H, W), dtype=np.uint8) if mask_rate > 0 else None
    for e in range(T):
        noise = rng.standard_normal((H, W), dtype=np.float32)
        if mask is not None:
            mask[e] = rng.random((H, W), dtype=np.float32) < np.float32(mask_rate)
        S = np.zeros((H, W), dtype=np.float64)
        for s in sources:
            x = s["x0"] + s["vx"] * times[e]
            y = s["y0"] + s["vy"] * times[e]
            x0, y0, g = _stamp(psf_sigma, r, x, y, s["flux"])
            ys0, xs0 = max(y0, 0), max(x0, 0)
            ys1, xs1 = min(y0 + g.shape[0], H), min(x0 + g.shape[1], W)
            if ys1 > ys0 and xs1 > xs0:
                S[ys0:ys1, xs0:xs1] += g[ys0 - y0:ys1 - y0, xs0 - x0:xs1 - x0]
        if unit_variance:
            var[e] = 1.0
            sci[e] = (S + noise.astype(np.float64)).astype(np.float32)
        else:
            v = sky + S
            var[e] = v.astype(np.float32)
            sci[e] = (S + np.sqrt(v) * noise).astype(np.float32)
    if vels is None:
        vels = np.zeros((1, 2), dtype=np.float32)
    return Stack(sci=sci, var=var, mask=mask, psf=psf, times=times,
                 vels=np.ascontiguousarray(vels, dtype=np.float32),
                 sources=sources, params=dict(params or {}), name=name)


def _source_speeds(W, H, sigma, t_max, lo=90.0, hi=500.0):
    """Source speed range, capped so that a whole track fits in small crops
    (a 256-px test image cannot hold a 500 px/day mover over two days)."""
    span = min(W, H) - 2 * (psf_size(sigma) // 2 + 2)
    vmax = min(hi, 0.9 * span / max(t_max, 1e-9))
    return (min(lo, 0.5 * vmax), vmax)


def _search_params(T, k, min_obs=None, sigmag=1):
    return dict(k=k, min_obs=default_min_obs(T) if min_obs is None else min_obs,
                sigmag=sigmag, q_lo=0.25, q_hi=0.75, coeff=0.7413, n_sigma=2.0)


def make_config(n: int, seed: Optional[int] = None, *, size=None,
                n_vel=None) -> Stack:
    """Named workloads.

    1: tiny plain search (64x64, T=5, one source, 16x16 grid, K=1).
    2: one DECam-CCD-shaped stack (2048 wide x 4096 high, T=26 over 3
       nights, 1% mask, PSF sigma 1.4 on 9x9, 50 sources, 128x128 grid, K=8).
    5: full-pipeline stack (4096x4096, T=60 over 5 nights, 2% mask, sigma 1.6
       on 11x11, 200 sources with SNR in [2, 10], 64x64 coarse grid).
    ``size=(W, H)`` and ``n_vel=(n_angles, n_speeds)`` shrink configurations
    2 and 5 for tests while keeping their cadence, PSF and noise recipe.
    """
    seed = CONFIG_SEED_BASE + n if seed is None else seed
    if n == 1:
        W, H = size or (64, 64)
        rng = np.random.Generator(np.random.PCG64(seed))
        t = np.sort(rng.uniform(0.0, 1.0, size=5))
        t = t - t[0]
        na, ns = n_vel or (16, 16)
        angles = 2.0 * math.pi * np.arange(na) / na
        speeds = np.linspace(0.0, 20.0, ns)
        src = [dict(x0=20.0, y0=30.0, vx=10.0, vy=5.0, flux=100.0, snr=None)]
        return make_stack(W, H, t, 1.0, seed=seed + 500, sources=src,
                          unit_variance=True, vels=velocity_grid(speeds, angles),
                          params=_search_params(5, 1, min_obs=4), name="c1")
    if n == 2:
        W, H = size or (2048, 4096)
        na, ns = n_vel or (128, 128)
        t = night_times(26, 3)
        angles = np.linspace(-math.pi / 6, math.pi / 6, na)
        speeds = np.linspace(90.0, 500.0, ns)
        nsrc = 50 if size is None else max(1, int(round(50 * W * H / (2048 * 4096))))
        return make_stack(W, H, t, 1.4, seed=seed, n_sources=nsrc,
                          snr_range=(3.0, 15.0), mask_rate=0.01,
                          speed_range=_source_speeds(W, H, 1.4, t.max()),
                          vels=velocity_grid(speeds, angles),
                          params=_search_params(26, 8), name="c2")
    if n == 5:
        W, H = size or (4096, 4096)
        na, ns = n_vel or (64, 64)
        t = night_times(60, 5)
        angles = np.linspace(-math.pi / 6, math.pi / 6, na)
        speeds = np.linspace(90.0, 500.0, ns)
        nsrc = 200 if size is None else max(1, int(round(200 * W * H / 4096 ** 2)))
        return make_stack(W, H, t, 1.6, seed=seed, n_sources=nsrc,
                          snr_range=(2.0, 10.0), mask_rate=0.02,
                          speed_range=_source_speeds(W, H, 1.6, t.max()),
                          vels=velocity_grid(speeds, angles),
                          params=_search_params(60, 8), name="c5")
    raise ValueError(f"no single-stack configuration {n}")


def make_batched_specs(num_stacks: int = 62, seed: int = 3000,
                       sizes=(512, 1024, 2048, 4096)) -> List[dict]:
    """Shapes of the batched workload: W and H drawn independently from
    ``sizes``, T uniform in [10, 30] over 3 nights, PSF sigma in [1, 2].
    Stack j's pixels are drawn from seed ``seed + j``."""
    rng = np.random.Generator(np.random.PCG64(seed - 1))
    out = []
    for j in range(num_stacks):
        W = int(rng.choice(sizes))
        H = int(rng.choice(sizes))
        T = int(rng.integers(10, 31))
        sigma = float(rng.uniform(1.0, 2.0))
        out.append(dict(W=W, H=H, T=T, sigma=sigma, seed=seed + j))
    return out


def make_batched_stack(spec: dict, n_vel=(64, 64), n_sources: int = 20) -> Stack:
    na, ns = n_vel
    angles = np.linspace(-math.pi / 6, math.pi / 6, na)
    speeds = np.linspace(90.0, 500.0, ns)
    t = night_times(spec["T"], 3)
    return make_stack(spec["W"], spec["H"], t, spec["sigma"], seed=spec["seed"],
                      n_sources=n_sources, snr_range=(3.0, 15.0),
                      speed_range=_source_speeds(spec["W"], spec["H"],
                                                 spec["sigma"], float(t.max())),
                      mask_rate=0.01,
                      vels=velocity_grid(speeds, angles),
                      params=_search_params(spec["T"], 8),
                      name=f"c3-{spec['seed']}")


def add_static_artifacts(st: Stack, n: int, seed: int, psf_sigma: float,
                         snr_range=(20.0, 60.0), run=(5, 9),
                         gap_days: float = 0.5) -> List[dict]:
    """Add ``n`` static artifacts to ``st.sci`` in place: each a PSF-shaped
    blob at a fixed sub-pixel position, present in a run of consecutive
    epochs of one night (``run`` epochs, at least 5: the intranight repeats
    of a differencing residual), with per-epoch matched-filter SNR drawn
    from ``snr_range``.  Nights are groups of epochs separated by more than
    ``gap_days``.  Returns the artifacts' descriptions."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T, H, W = st.sci.shape
    r = psf_size(psf_sigma) // 2
    s2 = float(np.sum(gaussian_psf(psf_sigma).astype(np.float64) ** 2))
    order = np.argsort(st.times)
    nights, cur = [], [int(order[0])]
    for a, b in zip(order[:-1], order[1:]):
        if st.times[b] - st.times[a] > gap_days:
            nights.append(cur)
            cur = []
        cur.append(int(b))
    nights.append(cur)
    out = []
    for _ in range(n):
        night = nights[int(rng.integers(0, len(nights)))]
        m = int(min(len(night), rng.integers(run[0], run[1] + 1)))
        first = int(rng.integers(0, len(night) - m + 1))
        epochs = night[first:first + m]
        x = float(rng.uniform(r + 1, W - r - 2))
        y = float(rng.uniform(r + 1, H - r - 2))
        snr = float(rng.uniform(*snr_range))
        flux = snr * math.sqrt(SKY / s2)
        x0, y0, g = _stamp(psf_sigma, r, x, y, flux)
        for e in epochs:
            st.sci[e, y0:y0 + g.shape[0], x0:x0 + g.shape[1]] += g.astype(np.float32)
        out.append(dict(x=x, y=y, epochs=epochs, snr=snr, flux=flux))
    return out


def tiny_stack(seed: int, W: int = 12, H: int = 10, T: int = 4, k: int = 3,
               n_vel: int = 6, mask_rate: float = 0.15, masked_fill=None,
               max_speed: float = 6.0) -> Stack:
    """Small random stack for brute-force checks: random times in [0, 2],
    random velocities, random per-pixel variance and a random mask.  Masked
    pixels can be overwritten with ``masked_fill`` (NaN, 1e30, ...) to check
    that masked data never reaches the planes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.sort(rng.uniform(0.0, 2.0, size=T))
    sci = rng.standard_normal((T, H, W)).astype(np.float32) * 3.0
    var = rng.uniform(0.5, 4.0, size=(T, H, W)).astype(np.float32)
    mask = (rng.random((T, H, W)) < mask_rate).astype(np.uint8)
    if masked_fill is not None:
        sci[mask != 0] = np.float32(masked_fill)
    sig = float(rng.uniform(0.6, 1.5))
    psf = gaussian_psf(sig, k)
    vels = rng.uniform(-max_speed, max_speed, size=(n_vel, 2)).astype(np.float32)
    return Stack(sci=sci, var=var, mask=mask, psf=psf, times=t, vels=vels,
                 sources=[], params=_search_params(T, 3, min_obs=1), name="tiny")
