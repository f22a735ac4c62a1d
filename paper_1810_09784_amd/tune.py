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


def autotune(spec, pm, dev, reps: int = 10, save: bool = True, verbose: bool = False, streams: int = 1,
             select=None) -> dict:
    """Time every candidate tile shape on this map; keep the fastest.

    streams = 1 times fh_hough launches one after the other on one stream (the
    latency of one map).  streams = 2 times two plans of the shape alternating
    over two streams, the throughput arrangement in which one launch's rank
    build runs beside the other's tiles; the best shape for it can differ
    (smaller work-groups leave no LDS for the rank build beside them).
    select = (sq_k, sq_x0, min_dk) times fh_hough_select with that selection
    instead, each call's candidates fetched after the next call is enqueued.
    Every candidate must produce the same map."""
    import torch
    from . import fh
    assert streams in (1, 2)
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    ref = None
    best = None
    results = []
    n_x0 = fh.Plan.from_spec(spec).n_x0
    outs = None
    sts = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(streams - 1)]
    for tile in candidates(n_x0, spec.n_k, spec.n_fft):
        try:
            plans = [fh.Plan.from_spec(spec, tile=tile) for _ in range(streams)]
        except fh.FHError:
            continue
        if outs is None:
            outs = [torch.empty((plans[0].n_k, plans[0].n_x0), dtype=torch.int32, device=dev) for _ in range(streams)]

        def run(n):
            for st in sts[1:]:
                st.wait_stream(sts[0])
            for q in range(n):
                j = q % streams
                if select is None:
                    fh.fh_hough(plans[j], rp, bn, outs[j], sts[j])
                    continue
                fh.fh_hough_select(plans[j], rp, bn, outs[j], *select, stream=sts[j])
                if q > 0:
                    fh.fh_select_results(plans[(q - 1) % streams], as_dicts=False)
            if select is not None:
                fh.fh_select_results(plans[(n - 1) % streams], as_dicts=False)
            for st in sts[1:]:
                sts[0].wait_stream(st)

        run(2 * streams)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run(reps * streams)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (reps * streams)
        if ref is None:
            ref = outs[0].clone()
        if not all(torch.equal(ref, o) for o in outs):
            raise RuntimeError(f"tile {plans[0].tile} gives a different map")
        results.append((ms, plans[0].tile))
        if verbose:
            print(f"  {ms:8.4f} ms  {plans[0].tile}", flush=True)
        if best is None or ms < best[0]:
            best = (ms, plans[0].tile)
        for p in plans:
            p.destroy()
    entry = {"tile": best[1], "ms": best[0], "n_candidates": len(results), "streams": streams,
             "timed": "fh_hough" if select is None else f"fh_hough_select{tuple(select)}"}
    if save:
        c = _load()
        c[key(spec, pm.n_peaks)] = entry
        with open(CACHE_OUT, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return entry


def main():
    """Tune the benchmark's workloads and write the cache: the large map for
    its timed step (fh_hough_select with 5 x 5 squares, two plans on two
    streams), the small map and the 48 batched maps for one launch at a time
    (their shapes serve per-map launches; a batch runs the library's own
    shapes, which suit its shared persistent launch better)."""
    import argparse
    import time
    import torch
    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--only", choices=("large", "small", "batched"), default=None)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    work = [("large", synth.cfg_single_large(), 2, (5, 5, 3)), ("small", synth.cfg_single_small(), 1, None)]
    work += [("batched", s, 1, None) for s in synth.cfg_batched()]
    for name, spec, streams, sel in work:
        if a.only and name != a.only:
            continue
        pm = synth.make_peakmap(spec)
        t = time.time()
        e = autotune(spec, pm, dev, reps=a.reps, streams=streams, select=sel)
        print(f"{spec.name}: {e['tile']} {e['ms']:.4f} ms of {e['n_candidates']} shapes, "
              f"{streams} stream(s), {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main()
