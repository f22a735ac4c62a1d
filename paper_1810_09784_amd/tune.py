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


# ------------------------------------------------------------- batches --
# A batch shares one persistent launch: one work-group size for every map, and
# each map's rows per tile decide how much LDS its tiles take, hence how many
# work-groups share a CU.  The batch is tuned as a whole: candidates are
# (work-group size, LDS budget of a tile's differential rows, time splits),
# each map's whole-FFT tile derived from them, and the objective is the time
# of the batch's graph launch.

BATCH_THREADS = (256, 512, 1024)
BATCH_TILE_KB = (12, 16, 20, 24, 28, 32, 40)
BATCH_TSPLIT = (16, 64)


def batch_key(specs, peak_counts) -> str:
    import hashlib
    h = hashlib.sha256("|".join(key(s, int(p)) for s, p in zip(specs, peak_counts)).encode()).hexdigest()
    return f"batch{len(specs)}_{h[:16]}"


def batch_tile(n_x0: int, n_k: int, threads: int, tile_kb: int, tsplit: int) -> dict:
    """A whole-FFT tile over all columns with as many rows (a power of two, at
    most 64 and n_k) as fit tile_kb KB of differential rows."""
    cols = min(n_x0, 8192)
    pitch = (cols + 1 + 3) // 4 * 4
    rows = max(1, min(64, tile_kb * 1024 // (pitch * 4)))
    rows = 1 << (rows.bit_length() - 1)
    return dict(mode=1, rows=min(rows, n_k), cols=cols, threads=threads, tsplit=tsplit)


def batch_candidates():
    return [None] + [dict(threads=t, tile_kb=kb, tsplit=ts) for t in BATCH_THREADS for kb in BATCH_TILE_KB
                     for ts in BATCH_TSPLIT]


def lookup_batch(specs, peak_counts) -> Optional[List[dict]]:
    e = _load().get(batch_key(specs, peak_counts))
    return [dict(t) for t in e["tiles"]] if e else None


def autotune_batch(specs, pms, dev, reps: int = 10, save: bool = True, verbose: bool = False,
                   candidates=None) -> dict:
    """Time the batch's graph launch for every candidate (None: the library's
    own shapes); every candidate must produce the same maps.  Maps that the
    library would read in windowed mode keep its own shape."""
    import torch
    from . import fh
    peaks = [(torch.from_numpy(p.row_ptr).to(dev), torch.from_numpy(p.bin).to(dev)) for p in pms]
    auto = [fh.Plan.from_spec(s) for s in specs]
    geo = [(p.n_x0, p.n_k, p.tile["mode"]) for p in auto]
    for p in auto:
        p.destroy()
    maps = [torch.empty((k, x), dtype=torch.int32, device=dev) for x, k, _ in geo]
    ref, best, n = None, None, 0
    for cand in (candidates if candidates is not None else batch_candidates()):
        tiles = [None if cand is None or mode != 1 else batch_tile(x, k, cand["threads"], cand["tile_kb"],
                                                                   cand["tsplit"]) for x, k, mode in geo]
        try:
            plans = [fh.Plan.from_spec(s, tile=t) for s, t in zip(specs, tiles)]
        except fh.FHError:
            continue
        b = fh.Batch(plans, peaks, maps)
        for _ in range(2):
            b.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        got = [m.clone() for m in maps]
        if ref is None:
            ref = got
        elif not all(torch.equal(a, c) for a, c in zip(ref, got)):
            raise RuntimeError(f"batch candidate {cand} gives different maps")
        if verbose:
            print(f"  {ms:8.4f} ms  {cand}", flush=True)
        n += 1
        if best is None or ms < best[0]:
            best = (ms, cand, [p.tile for p in plans])
        b.destroy()
        for p in plans:
            p.destroy()
    entry = {"tiles": best[2], "params": best[1], "ms": best[0], "n_candidates": n, "timed": "batch graph launch"}
    if save:
        c = _load()
        c[batch_key(specs, [p.n_peaks for p in pms])] = entry
        with open(CACHE_OUT, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
    return entry


def main():
    """Tune the benchmark's workloads and write the cache: the 48 batched maps
    as one batch (graph launch), the large map for its timed step
    (fh_hough_select with 5 x 5 squares, two plans on two streams), the small
    map and the 48 batched maps each for one launch at a time (their shapes
    serve per-map launches)."""
    import argparse
    import time
    import torch
    from . import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--only", choices=("large", "small", "batched", "batch"), default=None)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    if a.only in (None, "batch"):  # the 48 maps as one batch
        specs = synth.cfg_batched()
        pms = [synth.make_peakmap(s) for s in specs]
        t = time.time()
        e = autotune_batch(specs, pms, dev, reps=max(a.reps, 10), verbose=True)
        print(f"batch of {len(specs)}: {e['params']} {e['ms']:.4f} ms of {e['n_candidates']} candidates, "
              f"{time.time() - t:.1f} s", flush=True)
        if a.only == "batch":
            return
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
