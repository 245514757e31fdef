"""Coarse search, candidate extraction and adjoint refinement.

The paper searches a dense velocity grid and keeps the trajectories whose
filtered likelihood clears a threshold (Section 3.1, 3.2).  This driver
replaces the dense grid by a coarse one: it searches the coarse grid
(``search``), takes the global top-N result slots (``extract_top``), and
moves each candidate to a sub-pixel start and a real-valued velocity by
gradient ascent on the bilinear likelihood (``refine``: the adjoint kernel
plus Adam).  Every step runs in the HIP kernels of libkbm; this module only
sequences the calls and records per-stage times with HIP events.
"""
from __future__ import annotations

import torch

from . import (SearchParams, extract_top, extract_workspace_size, refine,
               search, search_batched)


def coarse_to_fine(psi, phi, times, vels, params: SearchParams, n_candidates: int,
                   lh_min: float = float("-inf"), steps: int = 50, lr_pos: float = 0.3,
                   stream=None):
    """Search ``vels`` (a coarse grid), extract the top ``n_candidates`` slots
    with L' >= lh_min, and refine them for ``steps`` Adam steps.

    Returns a dict: params [n][4] (x0, y0, vx, vy) after refinement, lh (the
    bilinear likelihood there, with each candidate's keep mask frozen from
    the search), grid_params / grid_lh / keep (the extracted grid hits), and
    stage times in ms (search, extract, refine) measured with HIP events."""
    s = torch.cuda.current_stream() if stream is None else stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
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
    p, lh = refine(psi, phi, times, cand["params"], keep=cand["keep"], steps=steps,
                   lr_pos=lr_pos, stream=stream)
    ev[3].record(s)
    ev[3].synchronize()
    return dict(params=p, lh=lh, grid_params=cand["params"], grid_lh=cand["lh"],
                keep=cand["keep"], results=res,
                ms=dict(search=ev[0].elapsed_time(ev[1]),
                        extract=ev[1].elapsed_time(ev[2]),
                        refine=ev[2].elapsed_time(ev[3])))
