"""Follow-up of candidates on synthetic peakmaps (Sec. V of the paper).

The paper's follow-up corrects the strain data for a candidate's phase and
re-analyses with longer FFTs; that needs raw data and stays out.  What runs
on peakmaps is kept:
  - an over-resolved Hough map around each candidate: the coarse cell's
    neighbourhood (+-3 bins, the coincidence window) re-gridded `over` times
    finer in x0 and k (the paper's example: 10), computed by the same
    transform with an explicit grid; all candidates of a map in one batch;
  - the drift correction and frequency projection: fh_project moves every
    peak by the candidate's power-law drift and gives the critical ratio of
    the candidate's bin in the projection.
"""
from __future__ import annotations

from typing import List, NamedTuple

import numpy as np


class RoiGrid(NamedTuple):
    x0_min: float
    dx0: float
    n_x0: int
    k: np.ndarray  # ascending, >= 0


def roi_grid(x0_c: float, k_c: float, dx0: float, dk: float, over: int = 10, half: int = 3) -> RoiGrid:
    """Cells of width dx0/over and dk/over covering [x0_c - half dx0, x0_c +
    half dx0) and [k_c - half dk, k_c + half dk), negative k rows dropped."""
    if over < 1 or half < 1 or not (dx0 > 0 and dk > 0):
        raise ValueError("bad ROI grid")
    m = 2 * half * over
    ks = k_c + (dk / over) * (np.arange(m, dtype=np.float64) - half * over)
    return RoiGrid(x0_c - half * dx0, dx0 / over, m, ks[ks >= 0.0])


def refine(dev, spec_like, row_ptr, bin_, cands, dx0: float, dk, over: int = 10, half: int = 3):
    """Over-resolved maps around candidates (dicts with x0 and k, as fh_select
    gives them) on one peakmap, all in one batch.  spec_like: n, tfft, f_min,
    f_max, n_fft.  dk: the coarse k bin size (scalar or per candidate).
    Returns per candidate (map, grid, refined x0, refined k, count)."""
    import torch
    from . import fh
    plans, grids_, maps = [], [], []
    dks = np.broadcast_to(np.asarray(dk, dtype=np.float64), (len(cands),))
    for c, d in zip(cands, dks):
        g = roi_grid(float(c["x0"]), float(c["k"]), dx0, float(d), over, half)
        plans.append(fh.Plan(spec_like.n, spec_like.tfft, spec_like.f_min, spec_like.f_max, spec_like.n_fft, g.k,
                             x0_min=g.x0_min, dx0=g.dx0, n_x0=g.n_x0))
        grids_.append(g)
        maps.append(torch.empty((len(g.k), g.n_x0), dtype=torch.int32, device=dev))
    best = []
    if plans:
        b = fh.Batch(plans, [(row_ptr, bin_)] * len(plans), maps)
        b.launch()
        # the best cell of every refined map on the GPU: the selection with one
        # square per map (largest count; ties: smallest row, then smallest column)
        best = b.select(1, 1, 1)
        b.destroy()
    out = []
    for g, m, cl in zip(grids_, maps, best):
        top = [c for c in cl if not c["second"]]
        if top:
            r, col, cnt = int(top[0]["row"]), int(top[0]["col"]), int(top[0]["count"])
        else:  # a flat map (no spread, so no candidate): every cell ties, the first wins
            r, col = 0, 0
            cnt = int(m[0, 0])
        out.append((m, g, g.x0_min + (col + 0.5) * g.dx0, float(g.k[r]), cnt))
    return out
