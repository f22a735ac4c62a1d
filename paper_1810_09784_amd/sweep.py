"""The full sweep: a search layout of many generalized FrequencyHough maps.

Every braking index n in {2, 2.5, ..., 7} x T_FFT in {2, 4, 8} s over 30
sub-bands of 64 Hz from 100 Hz (up to 2020 Hz), T_obs = 5 days.  A peakmap
per (band, T_FFT) is shared by the 11 braking indices (90 peakmaps, 990 maps);
each map has 256 uniform k rows on [0, k_max], k_max = (1/T_FFT^2)/f_min^n
(Sec. VI.B), and the x0 grid of Sec. VI.C.  Injections: 200 power-law
sources, each drawn into one (band, T_FFT) peakmap with its n from the grid,
f0 inside the band, k on one of the rows 2 .. n_k/2 - 1 of its map, and added
power a uniform in [amp_lo, amp_hi].

k_layout="paper" gives every map the geometric k grid of Sec. VI.B over the
spindown range of its T_FFT level of Sec. VI.D, fdot in [1/(2 T_FFT)^2,
1/T_FFT^2], instead of the uniform rows; injections then sit on rows of those
grids.

One run: all maps in one batched persistent launch (captured graph), the
plain selection (sq_k x sq_x0 squares, second candidate 3 rows away) on
every map in one batched pass, the tile CNN's scores of every 64 x 64 tile
and its top tiles, the selection's re-check of those tiles alone (squares and
statistics of the tile), and the detection efficiency of both pipelines (a
detection: a candidate with CR >= thr within 3 bins of the injection's true
cell in its own map).  Candidates
farther than 10 bins from every injection of their map count as noise.
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import grids as GR
from . import synth as S

N_VALUES = tuple(2.0 + 0.5 * i for i in range(11))
TFFTS = (2.0, 4.0, 8.0)
T_OBS = 5 * 86400.0
N_K = 256


def band_edges(n_bands: int = 30, f_start: float = 100.0, width: float = 64.0):
    return [(f_start + width * b, f_start + width * (b + 1)) for b in range(n_bands)]


def map_k(layout: str, n: float, tfft: float, lo: float, hi: float, n_k: int) -> np.ndarray:
    """k rows of one map (ascending)."""
    if layout == "uniform":
        return S.uniform_k((1.0 / tfft ** 2) / lo ** n, n_k)
    if layout == "paper":
        return GR.k_grid(n, tfft, lo, hi, 1.0 / (2.0 * tfft) ** 2, 1.0 / tfft ** 2)[0]
    raise ValueError("k_layout is 'uniform' or 'paper'")


class Sweep:
    """Inputs, plans and maps of the sweep, resident on the GPU."""

    def __init__(self, dev, seed: int = 5, n_values=N_VALUES, tffts=TFFTS, n_bands: int = 30, t_obs: float = T_OBS,
                 n_k: int = N_K, n_inj: int = 200, amp_lo: float = 1.0, amp_hi: float = 4.0, log=None,
                 k_layout: str = "uniform", groups=None):
        """groups: optional set of (band index, T_FFT index) to build, the others
        are left out (the injections are drawn for the whole sweep either way,
        so a group is built the same alone or with the rest)."""
        import torch
        from . import fh
        self.dev = dev
        self.seed = seed
        rng = np.random.default_rng(seed)
        self.bands = band_edges(n_bands)
        self.n_values, self.tffts = tuple(n_values), tuple(tffts)
        self.k_layout = k_layout
        # injections: (band, tfft index, n index, f0, k, amp, k row)
        inj = []
        for _ in range(n_inj):
            b = int(rng.integers(len(self.bands)))
            ti = int(rng.integers(len(self.tffts)))
            ni = int(rng.integers(len(self.n_values)))
            lo, hi = self.bands[b]
            n = self.n_values[ni]
            # on a k row of its map: a grid this coarse moves a track by many columns
            # per row over days, so off-row sources smear over the map
            ks = map_k(k_layout, n, self.tffts[ti], lo, hi, n_k)
            row = int(rng.integers(2, max(3, len(ks) // 2)))
            k = float(ks[row])
            f0 = float(rng.uniform(lo + 4.0, hi - 4.0))
            inj.append((b, ti, ni, f0, k, float(rng.uniform(amp_lo, amp_hi)), row))
        built = (lambda b, ti: True) if groups is None else (lambda b, ti: (b, ti) in groups)
        self.injections = [x for x in inj if built(x[0], x[1])]
        self.peakmaps = {}   # (band, ti) -> (row_ptr, bin)
        self.maps = []       # dicts: band, ti, ni, plan, hmap, peaks key, U
        self._index = {}     # (band, ti, ni) -> position in maps
        self.U = 0
        t = time.perf_counter()
        for b, (lo, hi) in enumerate(self.bands):
            for ti, tfft in enumerate(self.tffts):
                if not built(b, ti):
                    continue
                n_fft = int(t_obs / tfft)
                injs = [S.Injection(f0=f0, tau=1.0 / (k * (self.n_values[ni] - 1) * f0 ** (self.n_values[ni] - 1)),
                                    n=self.n_values[ni], amp=amp)
                        for (bb, tt, ni, f0, k, amp, _) in inj if bb == b and tt == ti]
                spec = S.MapSpec(f"b{b}t{tfft}", 3.0, tfft, lo, hi, n_fft, np.zeros(1), seed=seed * 100000 + b * 10 + ti,
                                 injections=injs)
                rp, bn, _ = S.gpu_peakmap(spec, dev)
                self.peakmaps[(b, ti)] = (rp, bn)
                P = int(bn.numel())
                for ni, n in enumerate(self.n_values):
                    kk = map_k(k_layout, n, tfft, lo, hi, n_k)
                    plan = fh.Plan(n, tfft, lo, hi, n_fft, kk)
                    hmap = torch.empty((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
                    self._index[(b, ti, ni)] = len(self.maps)
                    self.maps.append({"band": b, "ti": ti, "ni": ni, "n": n, "tfft": tfft, "f_min": lo, "f_max": hi,
                                      "n_fft": n_fft, "k": kk, "plan": plan, "hmap": hmap, "P": P})
                    self.U += P * len(kk)
        torch.cuda.synchronize()
        self.build_s = time.perf_counter() - t
        self.peaks_total = sum(int(bn.numel()) for _, bn in self.peakmaps.values())
        if log:
            log(f"sweep: {len(self.maps)} maps, {len(self.peakmaps)} peakmaps, {self.peaks_total:.3e} peaks, "
                f"U = {self.U:.3e} ({self.build_s:.1f} s to build)")
        self.batch = fh.Batch([m["plan"] for m in self.maps],
                              [self.peakmaps[(m["band"], m["ti"])] for m in self.maps],
                              [m["hmap"] for m in self.maps])

    def map_index(self, b, ti, ni):
        return self._index[(b, ti, ni)]

    def destroy(self):
        self.batch.destroy()


def time_batch(sw: Sweep, steps: int = 5, warmup: int = 2, stream=None):
    import torch
    for _ in range(warmup):
        sw.batch.launch(stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sw.batch.launch(stream)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_plain(sw: Sweep):
    import torch
    sw.batch.launch_plain()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sw.batch.launch_plain()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


TILE_SQ = (2, 1)  # squares of the learned pipeline's re-check inside a 64 x 64 tile


def _run_pipelines(sw: Sweep, net, sq, top_frac: float):
    """Launch the batch and select on every map (plain pipeline); with a
    network, score every map's tiles, take each map's top fraction and let the
    selection re-check those tiles alone, with the tiles' own squares and
    statistics (learned pipeline).  Returns (plain candidate records per map,
    learned candidate records per map or None, seconds of the selection,
    seconds of proposals and re-check, tiles scored)."""
    import torch
    from . import fh
    sw.batch.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cands = sw.batch.select(sq[0], sq[1], 3, as_dicts=False)  # every map in one batched pass
    t_sel = time.perf_counter() - t0
    if net is None:
        return cands, None, t_sel, 0.0, 0
    t0 = time.perf_counter()
    tops, n_tiles = [], 0
    for m in sw.maps:
        ta, tb = (m["plan"].n_k + 63) // 64, (m["plan"].n_x0 + 63) // 64
        tops.append(max(1, int(math.ceil(top_frac * ta * tb))))
        n_tiles += ta * tb
    _, best = fh.fh_batch_propose(net, sw.batch, tops)  # every map's tiles through the network at once
    req = [(mi, t) for mi, b in enumerate(best) for t in b]
    rc, counts, _ = sw.batch.select_tiles(req, TILE_SQ[0], TILE_SQ[1], 3)
    parts = [[] for _ in sw.maps]
    at = 0
    for (mi, _), c in zip(req, counts):
        parts[mi].append(rc[at:at + c])
        at += c
    learned = [np.concatenate(x) if x else rc[:0] for x in parts]
    return cands, learned, t_sel, time.perf_counter() - t0, n_tiles


def _truth(sw: Sweep):
    """Per map: the true cells (row, column) of its injections."""
    truth: Dict[int, List] = {}
    for (b, ti, ni, f0, k, amp, row) in sw.injections:
        mi = sw.map_index(b, ti, ni)
        m = sw.maps[mi]
        info = m["plan"].info
        col = (f0 ** (1.0 - m["n"]) - info.x0_min) / info.dx0
        truth.setdefault(mi, []).append((row, col))
    return truth


def evaluate(sw: Sweep, net=None, sq=(8, 8), top_frac: float = 0.1, thresholds=(4.0, 5.0, 6.0)):
    """The plain selection on every map and, with a network, the learned
    pipeline (its proposals re-checked by the selection); efficiencies of both
    and their noise candidates at each CR threshold."""
    cands, learned, t_sel, t_prop, n_tiles = _run_pipelines(sw, net, sq, top_frac)
    truth = _truth(sw)
    res = {"select_s": t_sel, "propose_s": t_prop, "tiles": n_tiles, "curves": []}
    noise_plain = {thr: 0 for thr in thresholds}
    noise_learn = {thr: 0 for thr in thresholds}
    det_plain = {thr: 0 for thr in thresholds}
    det_learn = {thr: 0 for thr in thresholds}

    def far(c, tr):
        return not tr or min(math.hypot(float(c["row"]) + 0.5 - r, float(c["col"]) + 0.5 - x) for (r, x) in tr) > 10.0

    def hit(cl, thr, r, x):
        return any(float(c["cr"]) >= thr and math.hypot(float(c["row"]) + 0.5 - r, float(c["col"]) + 0.5 - x) <= 3.0
                   for c in cl)

    for mi, cl in enumerate(cands):
        tr = truth.get(mi, [])
        lc = learned[mi] if learned is not None else []
        for thr in thresholds:
            noise_plain[thr] += sum(1 for c in cl if c["cr"] >= thr and far(c, tr))
            noise_learn[thr] += sum(1 for c in lc if c["cr"] >= thr and far(c, tr))
            for (r, x) in tr:
                det_plain[thr] += hit(cl, thr, r, x)
                det_learn[thr] += hit(lc, thr, r, x)
    n_inj = len(sw.injections)
    for thr in thresholds:
        res["curves"].append({"cr_thr": thr, "eff_plain": det_plain[thr] / n_inj,
                              "eff_learned": det_learn[thr] / n_inj if learned is not None else None,
                              "noise_cands_plain": noise_plain[thr],
                              "noise_cands_learned": noise_learn[thr] if learned is not None else None})
    return res


def map_maxima(sw: Sweep, net, sq=(8, 8), top_frac: float = 0.1) -> np.ndarray:
    """Per map: the largest CR of the plain selection's candidates and of the
    learned pipeline's (the re-check of the proposed tiles); -inf for none."""
    cands, learned, _, _, _ = _run_pipelines(sw, net, sq, top_frac)
    out = np.full((len(cands), 2), -np.inf)
    for mi, cl in enumerate(cands):
        if len(cl):
            out[mi, 0] = float(cl["cr"].max())
        if learned is not None and len(learned[mi]):
            out[mi, 1] = float(learned[mi]["cr"].max())
    return out


def evaluate_at_fap(dev, net, faps, n_noise_sweeps: int, seed: int, sw: Optional[Sweep] = None, sq=(8, 8),
                    top_frac: float = 0.1, amp_edges=(1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0), log=None, **kw) -> list:
    """Efficiency of both pipelines at fixed false-alarm probabilities per map.
    Noise-only sweeps (no injection, other seeds) give, per pipeline and per
    entry of `faps`, the smallest CR threshold whose exceedance by a map's
    largest candidate CR is at most that probability; an injection of `sw`
    counts as found when a candidate within 3 bins of its true cell (inside the
    proposed tiles, for the learned pipeline) reaches the pipeline's threshold.
    One record per entry of `faps`, with the efficiencies also binned by the
    injections' amplitude (`amp_edges`)."""
    from . import learn
    noise = []
    for q in range(n_noise_sweeps):
        nsw = Sweep(dev, seed=seed + 1000 + q, n_inj=0, **kw)
        noise.append(map_maxima(nsw, net, sq, top_frac))
        nsw.destroy()
        if log:
            log(f"noise sweep {q + 1}/{n_noise_sweeps}")
    noise = np.concatenate(noise, 0)
    own = sw is None
    if own:
        sw = Sweep(dev, seed=seed, **kw)
    cands, learned, _, _, _ = _run_pipelines(sw, net, sq, top_frac)
    # per injection: the largest CR near its true cell, of each pipeline's candidates
    best = np.full((len(sw.injections), 2), -np.inf)
    for i, (b, ti, ni, f0, k, amp, row) in enumerate(sw.injections):
        mi = sw.map_index(b, ti, ni)
        m = sw.maps[mi]
        info = m["plan"].info
        col = (f0 ** (1.0 - m["n"]) - info.x0_min) / info.dx0
        for q, cl in enumerate((cands[mi], learned[mi] if learned is not None else [])):
            for c in cl:
                if math.hypot(float(c["row"]) + 0.5 - row, float(c["col"]) + 0.5 - col) <= 3.0:
                    best[i, q] = max(best[i, q], float(c["cr"]))
    amps = np.array([inj[5] for inj in sw.injections])
    if own:
        sw.destroy()
    out = []
    for fap in faps:
        thr_p = learn.threshold_for_fap(noise[:, 0], fap)
        thr_l = learn.threshold_for_fap(noise[:, 1], fap)
        out.append({"fap_per_map": fap, "noise_maps": int(noise.shape[0]), "thr_plain": thr_p, "thr_learned": thr_l,
                    "fap_plain": float(np.mean(noise[:, 0] >= thr_p)),
                    "fap_learned": float(np.mean(noise[:, 1] >= thr_l)),
                    "injections": int(best.shape[0]), "eff_plain": float(np.mean(best[:, 0] >= thr_p)),
                    "eff_learned": float(np.mean(best[:, 1] >= thr_l)), "tiles_proposed_frac": top_frac,
                    "by_amp": []})
        for lo, hi in zip(amp_edges[:-1], amp_edges[1:]):
            sel = (amps >= lo) & (amps < hi)
            if sel.any():
                out[-1]["by_amp"].append({"amp_lo": lo, "amp_hi": hi, "n": int(sel.sum()),
                                          "eff_plain": float(np.mean(best[sel, 0] >= thr_p)),
                                          "eff_learned": float(np.mean(best[sel, 1] >= thr_l))})
    return out


class Checkpoint:
    """Per-map results of a sweep in a JSON-lines file, one record per map keyed
    by (n, T_FFT, f_min, f_max, seed).  Records are appended and flushed to disk
    one at a time; a last line cut short by a crash is dropped on reload."""

    def __init__(self, path: str):
        import json
        import os
        self.path = path
        self.done = {}
        good = 0
        if os.path.exists(path):
            with open(path, "rb") as f:
                data = f.read()
            at = 0
            for line in data.split(b"\n")[:-1]:  # the text after the last newline is incomplete
                at += len(line) + 1
                try:
                    rec = json.loads(line)
                except ValueError:
                    break
                if not isinstance(rec, dict) or "key" not in rec:
                    break
                self.done[self.key(*rec["key"])] = rec
                good = at
            if good != len(data):
                with open(path, "r+b") as f:
                    f.truncate(good)

    @staticmethod
    def key(n, tfft, f_min, f_max, seed):
        return (float(n), float(tfft), float(f_min), float(f_max), int(seed))

    def write(self, rec: dict):
        import json
        import os
        with open(self.path, "a") as f:
            f.write(json.dumps(rec) + "\n")
            f.flush()
            os.fsync(f.fileno())
        self.done[self.key(*rec["key"])] = rec


def run_resumable(dev, path: str, sq=(8, 8), min_dk: int = 3, cr_thr: float = 4.0, after_group=None, log=None,
                  **kw) -> int:
    """The sweep one (band, T_FFT) group of maps at a time (one batched launch
    and one batched selection per group), each map's result appended to the
    checkpoint file `path` as soon as its group is done: its candidates with
    CR >= cr_thr, the map's CRC-32 and total count, and its bad-peak count.
    Maps already in the file are skipped, so a run that stopped part-way
    continues where it stopped.  after_group(b, ti) is called after each group
    that was computed.  Returns the number of maps computed by this call."""
    import zlib
    import torch
    from . import fh
    ck = Checkpoint(path)
    seed = kw.get("seed", 5)
    bands = band_edges(kw.get("n_bands", 30))
    tffts = tuple(kw.get("tffts", TFFTS))
    n_values = tuple(kw.get("n_values", N_VALUES))
    computed = 0
    for b, (lo, hi) in enumerate(bands):
        for ti, tfft in enumerate(tffts):
            keys = [Checkpoint.key(n, tfft, lo, hi, seed) for n in n_values]
            if all(k in ck.done for k in keys):
                continue
            sw = Sweep(dev, groups={(b, ti)}, **kw)
            sw.batch.launch()
            torch.cuda.synchronize()
            cands = sw.batch.select(sq[0], sq[1], min_dk, cr_thr=cr_thr, as_dicts=False)
            for m, cl in zip(sw.maps, cands):
                key = Checkpoint.key(m["n"], m["tfft"], m["f_min"], m["f_max"], seed)
                if key in ck.done:
                    continue
                h = m["hmap"].cpu().numpy()
                ck.write({"key": list(key), "n_k": int(h.shape[0]), "n_x0": int(h.shape[1]),
                          "map_crc32": int(zlib.crc32(h.tobytes())), "map_sum": int(h.sum(dtype=np.int64)),
                          "bad_peaks": int(fh.fh_device_errors(m["plan"])),
                          "candidates": [[int(c["row"]), int(c["col"]), int(c["count"]), int(c["second"]),
                                          float(c["cr"])] for c in cl]})
                computed += 1
            sw.destroy()
            if log:
                log(f"sweep group band {b} T_FFT {tfft}: {len(sw.maps)} maps done")
            if after_group:
                after_group(b, ti)
    return computed


def main():
    import argparse
    import json
    import os
    import sys

    import torch
    from . import fh
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--bands", type=int, default=30)
    ap.add_argument("--weights", default=os.path.join(os.path.dirname(__file__), "trained", "tile_cnn_sweep.npy"))
    a = ap.parse_args()
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    sw = Sweep(dev, n_bands=a.bands, log=log)
    ms_b = time_batch(sw)
    ms_p = time_plain(sw)
    log(f"batched {ms_b:.3f} ms, plain {ms_p:.3f} ms")
    net = fh.CNN(max_batch=256)
    net.set_params(np.load(a.weights))
    ev = evaluate(sw, net)
    out = {"maps": len(sw.maps), "peakmaps": len(sw.peakmaps), "peaks": sw.peaks_total, "updates": sw.U,
           "ms_batched": ms_b, "ms_plain": ms_p, "updates_per_s_batched": sw.U / (ms_b * 1e-3),
           "updates_per_s_plain": sw.U / (ms_p * 1e-3), **ev}
    print(json.dumps(out))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
    sw.destroy()


if __name__ == "__main__":
    main()
