"""Autotuner for the Hough tile shape (rows per tile, columns per tile,
work-group size, whole-FFT or windowed peak reading, time splits).

`autotune` times candidate shapes with the library's own kernel on the GPU,
checks that every candidate produces the same map, and records the fastest in
a JSON cache keyed by the map's geometry; `lookup` reads the cache (None means
the library's automatic shape)."""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional

_PKG = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_PKG, "tune_gfx950.json")
CACHE_OUT = os.environ.get("FH_TUNE_OUT", CACHE)  # where autotune() writes
_cache: Optional[Dict[str, dict]] = None


def key(spec, n_peaks: int) -> str:
    dens = n_peaks / max(1, spec.n_fft * spec.n_f)
    return f"nf{spec.n_f}_k{spec.n_k}_fft{spec.n_fft}_n{spec.n:g}_T{spec.tfft:g}_fmin{spec.f_min:g}_d{dens:.3f}"


def _load() -> Dict[str, dict]:
    global _cache
    if _cache is None:
        _cache = {}
        if os.path.exists(CACHE):
            with open(CACHE) as f:
                _cache = json.load(f)
    return _cache


def lookup(spec, n_peaks: int) -> Optional[dict]:
    e = _load().get(key(spec, n_peaks))
    return dict(e["tile"]) if e else None


def candidates(n_x0: int, n_k: int, n_fft: int) -> List[dict]:
    out = [None]
    if n_x0 <= 8192:
        for rows in (1, 2, 4, 8, 16, 32, 64):
            if rows > n_k:
                continue
            for ts in (1, 2, 4, 8, 16, 32):
                if ts > n_fft:
                    continue
                tiles = ((n_k + rows - 1) // rows) * ts
                if tiles < 128 or tiles > 65536:
                    continue
                for th in (256, 512):
                    out.append(dict(mode=1, rows=rows, cols=n_x0, threads=th, tsplit=ts))
    if n_x0 > 1024:
        for ntx in (1, 2, 3, 4, 6, 8, 12):
            cols = (n_x0 + ntx - 1) // ntx
            if cols > 40000:
                continue
            for rows in (1, 2):
                for th in (256, 512, 1024):
                    for ts in (16, 64, 256):
                        out.append(dict(mode=2, rows=rows, cols=cols, threads=th, tsplit=ts))
    return out


def autotune(spec, pm, dev, reps: int = 10, save: bool = True, verbose: bool = False) -> dict:
    """Time every candidate tile shape on this map; keep the fastest."""
    import torch
    from . import fh
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    ref = None
    best = None
    results = []
    n_x0 = fh.Plan.from_spec(spec).n_x0
    for tile in candidates(n_x0, spec.n_k, spec.n_fft):
        try:
            plan = fh.Plan.from_spec(spec, tile=tile)
        except fh.FHError:
            continue
        out = torch.empty((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
        for _ in range(2):
            fh.fh_hough(plan, rp, bn, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fh.fh_hough(plan, rp, bn, out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if ref is None:
            ref = out.clone()
        elif not torch.equal(ref, out):
            raise RuntimeError(f"tile {plan.tile} gives a different map")
        results.append((ms, plan.tile))
        if verbose:
            print(f"  {ms:8.4f} ms  {plan.tile}", flush=True)
        if best is None or ms < best[0]:
            best = (ms, plan.tile)
        plan.destroy()
    entry = {"tile": best[1], "ms": best[0], "n_candidates": len(results)}
    if save:
        c = _load()
        c[key(spec, pm.n_peaks)] = entry
        with open(CACHE_OUT, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return entry
