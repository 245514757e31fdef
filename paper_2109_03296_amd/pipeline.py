"""Coarse search, candidate extraction and adjoint refinement.

The paper searches a dense velocity grid and keeps the trajectories whose
filtered likelihood clears a threshold (Section 3.1, 3.2).  This driver
replaces the dense grid by a coarse one: it searches the coarse grid
(``search``), takes the global top-N result slots (``extract_top``), and
moves each candidate to a sub-pixel start and a real-valued velocity by
gradient ascent on the bilinear likelihood (``refine``: the adjoint kernel
plus Adam).  ``known_objects`` evaluates a given list of trajectories
(targeted mode: the search's filtered likelihood, then the median-stamp
moment cut, Section 3.3).  Every step runs in the HIP kernels of libkbm; this
module only sequences the calls and records per-stage times with HIP events.
"""
from __future__ import annotations

import torch

from . import (SearchParams, detect, extract_top, extract_workspace_size, refine,
               score_trajectories, search, search_batched, stamps)


def coarse_to_fine(psi, phi, times, vels, params: SearchParams, n_candidates: int,
                   lh_min: float = float("-inf"), steps: int = 50, lr_pos: float = 0.3,
                   stream=None):
    """Search ``vels`` (a coarse grid), extract the top ``n_candidates`` slots
    with L' >= lh_min, refine them for ``steps`` Adam steps, and score the
    refined trajectories with the search's filtered likelihood.

    The refinement ascends the bilinear likelihood over all usable epochs:
    a keep mask frozen at a coarse grid hit would hide the signal (there the
    epochs that line up with a source are the outliers the filter drops).
    Returns a dict: params [n][4] (x0, y0, vx, vy) after refinement; lh, keep,
    n_obs (the search's L' of the refined trajectories, from
    score_trajectories); lh_bilinear (the refined objective);
    grid_params / grid_lh / grid_keep (the extracted grid hits); and stage
    times in ms (search, extract, refine, score) from HIP events."""
    s = torch.cuda.current_stream() if stream is None else stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    ev[0].record(s)
    T = psi.shape[0]
    item = dict(psi=psi, phi=phi, times=times, vels=vels, params=params)
    if T <= 32 and params.k <= 8:
        res = search_batched([item], stream=stream, persistent=True)[0]
    else:
        res = search(psi, phi, times, vels, params, stream=stream)
    ev[1].record(s)
    Hr, Wr, k = res["lh"].shape
    ws = torch.empty(max(extract_workspace_size(Hr, Wr, k, len(vels)), 1),
                     dtype=torch.uint8, device=psi.device)
    origin = (params.region[0], params.region[1]) if params.region else (0, 0)
    cand = extract_top(res, vels, n_candidates, lh_min, region_origin=origin,
                       workspace=ws, stream=stream)
    ev[2].record(s)
    p, lh_bil = refine(psi, phi, times, cand["params"], keep=None, steps=steps,
                       lr_pos=lr_pos, stream=stream)
    ev[3].record(s)
    sc = score_trajectories(psi, phi, times, p, params, want_lh_raw=False, stream=stream)
    ev[4].record(s)
    ev[4].synchronize()
    return dict(params=p, lh=sc["lh"], keep=sc["keep"], n_obs=sc["n_obs"],
                lh_bilinear=lh_bil, grid_params=cand["params"], grid_lh=cand["lh"],
                grid_keep=cand["keep"], results=res,
                ms=dict(search=ev[0].elapsed_time(ev[1]),
                        extract=ev[1].elapsed_time(ev[2]),
                        refine=ev[2].elapsed_time(ev[3]),
                        score=ev[3].elapsed_time(ev[4])))


def known_objects(sci, var, mask, psi, phi, times, params, search_params: SearchParams,
                  lh_min: float = 10.0, radius: int = 10, stream=None):
    """Targeted mode: evaluate the given linear trajectories ``params`` [n][4]
    (x0, y0, vx, vy; float32, real-valued starts) with the search's filtered
    likelihood (``score_trajectories``), then coadd median stamps over the
    kept epochs and apply the central-moment cut (``stamps``).  A trajectory
    is detected when its n_obs >= min_obs, L' >= lh_min and its stamp passes
    the cut.  Returns a dict: lh, flux, keep, n_obs, moments, stamp_pass,
    detected (bool [n]) and stage times in ms (score, stamps)."""
    s = torch.cuda.current_stream() if stream is None else stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    prm = params.contiguous()
    ev[0].record(s)
    sc = score_trajectories(psi, phi, times, prm, search_params, want_lh_raw=False,
                            stream=stream)
    ev[1].record(s)
    st = stamps(sci, var, mask, times, prm, keep=sc["keep"], radius=radius,
                want_coadd=False, stream=stream)
    ev[2].record(s)
    ev[2].synchronize()
    det = detect(sc["lh"], sc["n_obs"], st["pass_u8"], search_params.min_obs, lh_min,
                 stream=stream)
    return dict(lh=sc["lh"], flux=sc["flux"], keep=sc["keep"], n_obs=sc["n_obs"],
                moments=st["moments"], stamp_pass=st["passed"], detected=det,
                ms=dict(score=ev[0].elapsed_time(ev[1]), stamps=ev[1].elapsed_time(ev[2])))
