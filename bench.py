#!/usr/bin/env python3
"""Benchmark of the generalized FrequencyHough hot path on one MI355X.

Workload: the large single map (n = 3, 200-1200 Hz, T_FFT = 4 s, 43200 FFTs =
2 days, 1024 k rows on [0, k_max], 84000 x0 columns, ~1.3e7 peaks of seeded
Exp(1) noise with 20 injections).  One step = the whole hot path on that
peakmap, inputs resident in HBM: fh_hough_select, that is peak ingest (rank
structure), the Hough transform into the differential LDS tiles with the
prefix sums, the map store and the selection's row pass in one kernel, then
the split-tile pass and the square reduction, and the host's CR finish of the
candidates.  The timed steps alternate two plans (two map buffers) on two
streams, so consecutive steps overlap on the GPU; the unfused path (fh_hough
then fh_select), serial and pipelined, is reported beside it.

Metric: FH Hough updates/s, an update being one (peak, k-row) pair, counted
over all P * n_k pairs.  Also reported: the batched persistent launch over the
48 uneven maps against the same maps launched one by one, the 990-map sweep,
the CNN, the search-layout steps, the roofline of the dominant kernel, and the
oracle timed on the host cores.

Prints one JSON line on stdout; progress goes to stderr."""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0  # dense matrix cores
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_k_queue_large_map.md")
BATCH_TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_k_queue_batch48.md")
KERNEL_SOURCES = ("paper_1810_09784_amd/csrc/fh_hough.hip", "paper_1810_09784_amd/csrc/fh_plan.cpp",
                  "paper_1810_09784_amd/csrc/fh_internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--cnn-only", action="store_true",
                    help="only the tile CNN section (forward, proposals' forward, training step), for profiling")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the 48-map batch's graph launches (no per-map launches, no oracle): for profiling")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 990-map sweep and the search-layout extras")
    ap.add_argument("--cpu-rows", type=int, default=0, help="k rows of the oracle sample (0: the whole map)")
    ap.add_argument("--fap-sweeps", type=int, default=30,
                    help="noise-only sweeps that calibrate the sweep's fixed-FAP thresholds (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter scale for HBM traffic)")
    return ap.parse_args()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_PROFILE):
    """HBM bytes per launch of a tile kernel from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when the kernel sources
    changed since the counters were taken."""
    import re
    try:
        with open(path) as f:
            txt = f.read()
    except OSError:
        return None
    m_b = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", txt, re.M)
    m_h = re.search(r"^kernel_sources_sha256:\s*([0-9a-f]{64})", txt, re.M)
    if not (m_b and m_h) or m_h.group(1) != kernel_source_hash():
        return None
    return int(m_b.group(1))


def machine():
    """The host and GPU the line was measured on."""
    import torch
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    p = torch.cuda.get_device_properties(0)
    return {"gpu": p.name, "gpu_arch": getattr(p, "gcnArchName", ""), "gpu_cus": p.multi_processor_count,
            "gpu_mem_gib": round(p.total_memory / 2**30, 1), "host_cpu": cpu,
            "host_threads": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}


def timed(fn, K, W, stream):
    import torch
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(K):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K


def run_sweep(fh, synth, dev, stream, cands_large, spec, plan, rp, bn, K, check_oracle, fap_sweeps=0):
    """The 990-map sweep (batched vs per-map launches, selection, CNN proposals,
    detection efficiency) and timings of the search-layout steps: a map on the
    paper's geometric k grid, coincidences of the sweep's candidates, the
    follow-up projection and over-resolved maps of the large map's candidates."""
    import math
    import numpy as np
    import torch
    from paper_1810_09784_amd import followup, grids, sweep
    t = time.perf_counter()
    sw = sweep.Sweep(dev, log=log)
    ms_b = sweep.time_batch(sw, steps=K, warmup=2, stream=stream)
    ms_p = sweep.time_plain(sw)
    net = fh.CNN(max_batch=256)
    net.set_params(np.load(os.path.join(ROOT, "paper_1810_09784_amd", "trained", "tile_cnn_sweep.npy")))
    ev = sweep.evaluate(sw, net)
    # one whole pass of the 990-map workload, wall clock: the batched Hough
    # launch, the selection on every map, the proposals on every map's tiles and
    # the selection's re-check of the proposed tiles (median of 3 after a warm-up)
    sweep._run_pipelines(sw, net, (8, 8), 0.1)
    walls = []
    for _ in range(3):
        torch.cuda.synchronize()
        t_w = time.perf_counter()
        sweep._run_pipelines(sw, net, (8, 8), 0.1)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t_w)
    wall_s = sorted(walls)[1]
    log(f"sweep: batched {ms_b:.3f} ms, plain {ms_p:.3f} ms, selection {ev['select_s']:.2f} s, "
        f"proposals {ev['propose_s']:.2f} s, whole pass {wall_s:.3f} s")
    at_fap = None
    if fap_sweeps > 0:
        # both pipelines at fixed false-alarm probabilities per map: thresholds from the
        # largest candidate CR of noise-only sweeps (other seeds), then this sweep's
        # injections scored at them (10% of the tiles proposed for the learned one)
        t0 = time.perf_counter()
        at_fap = sweep.evaluate_at_fap(dev, net, [0.1, 0.01, 0.001], fap_sweeps, 5, sw=sw)
        for r in at_fap:
            r.pop("by_amp", None)
        log(f"sweep: fixed-FAP efficiencies from {fap_sweeps} noise sweeps in {time.perf_counter() - t0:.1f} s: " +
            ", ".join(f"FAP {r['fap_per_map']:g}: plain {r['eff_plain']:.3f}, learned {r['eff_learned']:.3f}"
                      for r in at_fap))
    parity = sweep_parity(sw, seed=51) if check_oracle else None
    sweep_out = {"workload": "11 n (2..7) x T_FFT {2,4,8} s x 30 bands of 64 Hz from 100 Hz, 5 days, 256 k rows; "
                             "200 injections",
                 "maps": len(sw.maps), "peakmaps": len(sw.peakmaps), "peaks": sw.peaks_total,
                 "updates_per_launch": sw.U, "ms_batched": round(ms_b, 4), "ms_plain": round(ms_p, 4),
                 "updates_per_s_batched": sw.U / (ms_b * 1e-3), "updates_per_s_plain": sw.U / (ms_p * 1e-3),
                 "speedup_vs_plain": round(ms_p / ms_b, 3), "select_s": round(ev["select_s"], 3),
                 "propose_s": round(ev["propose_s"], 3), "tiles_scored": ev["tiles"],
                 "pipeline_wall_s": round(wall_s, 4),
                 "pipeline": "one pass, wall clock: batched Hough launch, selection on every map (8 x 8 squares), "
                             "CNN proposals on every tile, re-check of the top 10% of each map's tiles",
                 "efficiency": ev["curves"], "efficiency_at_fap": at_fap, "parity_vs_oracle": parity,
                 "note": "tile CNN trained on maps of this geometry drawn with other seeds (tile_cnn_sweep.npy)"}
    if parity:
        sweep_out.update(in_grid_pairs=parity["in_grid_pairs"],
                         in_grid_pairs_per_s_batched=parity["in_grid_pairs"] / (ms_b * 1e-3),
                         in_grid_pairs_per_s_plain=parity["in_grid_pairs"] / (ms_p * 1e-3))
    sw_paper = run_sweep_paper_k(fh, dev, stream, K, check_oracle)
    # coincidences: the sweep's candidates against a second draw of the same maps'
    # candidates is not available, so the list is joined with itself moved by one bin
    cl = sw.batch.select(8, 8, 3)
    pts, off = [], [0]
    for m, c in zip(sw.maps, cl):
        dk = float(m["k"][1] - m["k"][0])
        pts += [(x["x0"], x["k"], m["plan"].info.dx0, dk) for x in c]
        off.append(len(pts))
    A = torch.tensor(pts, dtype=torch.float64, device=dev)
    B = A.clone()
    B[:, 0] += B[:, 2]
    offs = torch.tensor(off, dtype=torch.int32, device=dev)
    fh.fh_coincide(offs, A, offs, B)
    ms_c = timed(lambda: fh.fh_coincide(offs, A, offs, B), 5, 1, stream)
    sw.destroy()
    # the paper's geometric k grid on the small band (n = 5, 500-600 Hz, T_FFT = 2 s)
    tg = 2.0
    ks, _ = grids.k_grid(5.0, tg, 500.0, 600.0, 1e-3 / tg ** 2, 1.0 / tg ** 2)
    spec_g = synth.MapSpec("paper-grid", 5.0, tg, 500.0, 600.0, 7200, ks, seed=1,
                           injections=synth.cfg_single_small().injections)
    pm_g = synth.make_peakmap(spec_g)
    plan_g = fh.Plan.from_spec(spec_g)
    rpg, bng = torch.from_numpy(pm_g.row_ptr).to(dev), torch.from_numpy(pm_g.bin).to(dev)
    hg = torch.empty((plan_g.n_k, plan_g.n_x0), dtype=torch.int32, device=dev)
    ms_g = timed(lambda: fh.fh_hough(plan_g, rpg, bng, hg, stream), K, 2, stream)
    grid_work = {}
    if check_oracle:
        from oracle import hough as oracle
        d_g = oracle.Desc.from_spec(spec_g)
        rows_g = np.arange(len(ks), dtype=np.int32)
        _, tot_g, pairs_g = oracle.rows_checked(d_g, pm_g.row_ptr, pm_g.bin, rows_g, with_map=False)
        ok_g = bool(np.array_equal(hg.sum(dim=1, dtype=torch.int64).cpu().numpy(), tot_g))
        grid_work = {"in_grid_pairs": int(pairs_g.sum()), "in_grid_pairs_per_s": int(pairs_g.sum()) / (ms_g * 1e-3),
                     "row_totals_equal_oracle": ok_g}
        assert ok_g, "paper-grid map row totals differ from the oracle"
    # follow-up of the large map's candidates: projections and over-resolved maps
    lst = cands_large["list"]
    f0t = torch.tensor([float(c["f0"]) for c in lst], dtype=torch.float64, device=dev)
    kt = torch.tensor([float(c["k"]) for c in lst], dtype=torch.float64, device=dev)
    ms_proj = timed(lambda: fh.fh_project(plan, rp, bn, f0t, kt, w=40, guard=2), 3, 1, stream)
    t_roi = time.perf_counter()
    roi = followup.refine(dev, spec, rp, bn, [dict(x0=float(c["x0"]), k=float(c["k"])) for c in lst], plan.info.dx0,
                          float(spec.k[1] - spec.k[0]))
    s_roi = time.perf_counter() - t_roi
    layout = {"paper_k_grid_map": {"workload": "n=5, 500-600 Hz, T_FFT=2 s, 7200 FFTs, geometric k grid "
                                               "(fdot 1e-3..1 x 1/T_FFT^2)", "k_rows": int(len(ks)),
                                   "ms": round(ms_g, 4), "updates_per_s": pm_g.n_peaks * len(ks) / (ms_g * 1e-3),
                                   **grid_work},
              "coincide": {"points": len(pts), "segments": len(off) - 1, "ms": round(ms_c, 4)},
              "project": {"candidates": len(lst), "peaks": int(bn.numel()), "ms": round(ms_proj, 4),
                          "peak_moves_per_s": len(lst) * int(bn.numel()) / (ms_proj * 1e-3)},
              "roi_refine": {"candidates": len(roi), "cells_each": 60 * 60, "s_incl_plans": round(s_roi, 3)}}
    log(f"layout: paper grid {ms_g:.3f} ms ({len(ks)} rows), coincide {ms_c:.3f} ms ({len(pts)} points), "
        f"project {ms_proj:.3f} ms, ROI refine {s_roi:.2f} s")
    layout["sweep_paper_k_grids"] = sw_paper
    return sweep_out, layout


def run_cnn(fh, dev, stream, B=256, reps=20):
    """Forward passes and training steps of the tile CNN on B random tiles:
    throughput against the BF16 dense matrix-core peak (about 492 MFLOP per
    tile forward, 3x that per training tile)."""
    import numpy as np
    import torch
    net = fh.CNN(max_batch=B)
    rng = np.random.default_rng(1)
    net.set_params(rng.normal(0.0, 0.05, net.n_params).astype(np.float32))
    x = torch.from_numpy(rng.normal(0.0, 1.0, (B, 64, 64)).astype(np.float32)).to(dev).to(torch.bfloat16)
    lab = torch.from_numpy((rng.random(B) < 0.5).astype(np.float32)).to(dev)
    fwd = timed(lambda: net.forward(x, stream=stream), reps, 3, stream)
    sco = timed(lambda: net.scores(x, stream=stream), reps, 3, stream)  # the proposals' forward

    def train():
        net.forward(x, stream=stream)
        net.backward(lab, stream=stream)
        net.step(1e-3, stream=stream)

    trn = timed(train, reps // 2, 2, stream)
    net.destroy()
    f_fwd = 492.0e6 * B
    tf_fwd, tf_trn = f_fwd / (fwd * 1e-3) / 1e12, 3 * f_fwd / (trn * 1e-3) / 1e12
    tf_sco = f_fwd / (sco * 1e-3) / 1e12
    log(f"cnn: forward {fwd:.3f} ms / {B} tiles ({tf_fwd:.0f} TFLOP/s), proposals' forward {sco:.3f} ms "
        f"({tf_sco:.0f} TFLOP/s), training step {trn:.3f} ms ({tf_trn:.0f} TFLOP/s)")
    return {"tiles_per_batch": B, "forward_ms": round(fwd, 4), "forward_tiles_per_s": B / (fwd * 1e-3),
            "scores_ms": round(sco, 4), "scores_tiles_per_s": B / (sco * 1e-3), "scores_tflops": round(tf_sco, 1),
            "scores_mfma_frac": round(tf_sco / BF16_PEAK_TFLOPS, 4),
            "forward_tflops": round(tf_fwd, 1), "train_step_ms": round(trn, 4), "train_tflops": round(tf_trn, 1),
            "peak_tflops": BF16_PEAK_TFLOPS, "forward_mfma_frac": round(tf_fwd / BF16_PEAK_TFLOPS, 4),
            "train_mfma_frac": round(tf_trn / BF16_PEAK_TFLOPS, 4), **_mfma_measured(tf_fwd, tf_trn)}


def _mfma_measured(tf_fwd, tf_trn):
    from paper_1810_09784_amd import ceilings
    ceil = ceilings.load()
    if not ceil:
        return {}
    m = ceil["tests"]["mfma_bf16_16x16x32"]["tflops"]
    return {"measured_peak_tflops": m, "forward_frac_measured": round(tf_fwd / m, 4),
            "train_frac_measured": round(tf_trn / m, 4)}


def sweep_parity(sw, seed, pct=10):
    """Every map of a sweep against the oracle: a seeded sample of at least
    `pct` percent of its rows compared cell by cell with the oracle's direct counts,
    and every row's total (sum of its peaks' clipped interval widths) against
    the GPU map's row sum; also the (peak, row) pairs that land in the grid."""
    import numpy as np
    import torch
    from oracle import hough as oracle
    t0 = time.perf_counter()
    rng = np.random.default_rng(seed)
    key, rph, bnh = None, None, None
    n_rows = n_cmp = n_maps_ok = 0
    pairs = 0
    rows_equal = totals_equal = True
    for m in sw.maps:
        if (m["band"], m["ti"]) != key:
            key = (m["band"], m["ti"])
            rp_d, bn_d = sw.peakmaps[key]
            rph, bnh = rp_d.cpu().numpy(), bn_d.cpu().numpy()
        n_k = m["plan"].n_k
        d = oracle.Desc(m["n"], m["tfft"], m["f_min"], m["f_max"], m["n_fft"], m["k"])
        sample = np.sort(rng.choice(n_k, max(1, -(-n_k * pct // 100)), replace=False)).astype(np.int32)
        ref_rows, _, _ = oracle.rows_checked(d, rph, bnh, sample)
        got_rows = m["hmap"][torch.from_numpy(sample).long().to(m["hmap"].device)].cpu().numpy()
        _, ref_tot, ref_pairs = oracle.rows_checked(d, rph, bnh, np.arange(n_k, dtype=np.int32), with_map=False)
        got_tot = m["hmap"].sum(dim=1, dtype=torch.int64).cpu().numpy()
        ok_r = bool(np.array_equal(got_rows, ref_rows))
        ok_t = bool(np.array_equal(got_tot, ref_tot))
        rows_equal &= ok_r
        totals_equal &= ok_t
        n_maps_ok += ok_r and ok_t
        n_rows += n_k
        n_cmp += len(sample)
        pairs += int(ref_pairs.sum())
    out = {"checked": f"all {len(sw.maps)} maps: a seeded {pct}% sample of each map's rows cell by cell "
                      f"({n_cmp} rows) and every row's total ({n_rows} rows) against the oracle",
           "rows_compared": n_cmp, "rows_with_totals": n_rows, "maps_equal": n_maps_ok,
           "sampled_rows_equal": rows_equal, "row_totals_equal": totals_equal, "equal": rows_equal and totals_equal,
           "in_grid_pairs": pairs, "oracle_s": round(time.perf_counter() - t0, 1)}
    log(f"sweep parity: {n_maps_ok}/{len(sw.maps)} maps equal ({n_cmp} sampled rows, {n_rows} row totals), "
        f"{pairs:.4e} in-grid pairs, {out['oracle_s']} s")
    assert out["equal"], "sweep maps differ from the oracle"
    return out


def run_sweep_paper_k(fh, dev, stream, K, check_oracle):
    """The sweep's 990 maps on the paper's k layout: each map on the geometric k
    grid of Sec. VI.B over its T_FFT level's spindown range [1/(2 T_FFT)^2,
    1/T_FFT^2] (Sec. VI.D) instead of 256 uniform rows."""
    import numpy as np
    from paper_1810_09784_amd import sweep
    sw = sweep.Sweep(dev, log=log, k_layout="paper")
    rows = [m["plan"].n_k for m in sw.maps]
    ms_b = sweep.time_batch(sw, steps=K, warmup=1, stream=stream)
    ev = sweep.evaluate(sw, None)
    log(f"sweep (paper k grids): {sum(rows)} rows ({min(rows)}-{max(rows)} per map), batched {ms_b:.3f} ms, "
        f"selection {ev['select_s']:.2f} s")
    parity = sweep_parity(sw, seed=52) if check_oracle else None
    out = {"workload": "the 990 sweep maps, each on the geometric k grid of its T_FFT level "
                       "(fdot 1/(2 T_FFT)^2 .. 1/T_FFT^2); 200 injections on grid rows",
           "k_rows": int(sum(rows)), "rows_per_map": [int(min(rows)), int(max(rows))],
           "updates_per_launch": sw.U, "ms_batched": round(ms_b, 4), "updates_per_s_batched": sw.U / (ms_b * 1e-3),
           "select_s": round(ev["select_s"], 3), "efficiency_plain": [
               {k: c[k] for k in ("cr_thr", "eff_plain", "noise_cands_plain")} for c in ev["curves"]],
           "parity_vs_oracle": parity}
    if parity:
        out.update(in_grid_pairs=parity["in_grid_pairs"],
                   in_grid_pairs_per_s_batched=parity["in_grid_pairs"] / (ms_b * 1e-3))
    sw.destroy()
    return out


def run_batched(fh, synth, tune, ceilings, dev, stream, K, W, check_oracle, plain=True):
    """The 48 uneven maps as one persistent graph launch, against the same maps
    launched one by one (fh_hough per map with its autotuned shape); every map
    checked against the oracle, with the in-grid pair count of each."""
    import numpy as np
    import torch
    out = {}
    t = time.perf_counter()
    specs = synth.cfg_batched()
    # each path with its own best shapes: the batch with those tuned for its shared
    # persistent launch, the per-map launches with the shapes the autotuner found
    # for each map alone (python -m paper_1810_09784_amd.tune)
    plans, plans_t, peaks, maps, Ub = [], [], [], [], 0
    pms = [synth.make_peakmap(s) for s in specs]
    # the batch's shapes tuned for its graph launch as a whole (tune.autotune_batch),
    # else the library's own
    tiles_b = tune.lookup_batch(specs, [p.n_peaks for p in pms])
    for i, (s, p) in enumerate(zip(specs, pms)):
        pl = fh.Plan.from_spec(s, tile=tiles_b[i] if tiles_b else None)
        plans.append(pl)
        plans_t.append(fh.Plan.from_spec(s, tile=tune.lookup(s, p.n_peaks)))
        peaks.append((torch.from_numpy(p.row_ptr).to(dev), torch.from_numpy(p.bin).to(dev)))
        maps.append(torch.empty((pl.n_k, pl.n_x0), dtype=torch.int32, device=dev))
        Ub += p.n_peaks * pl.n_k
    batch = fh.Batch(plans, peaks, maps)
    log(f"batched: {len(specs)} maps, U = {Ub:.4e} ({time.perf_counter() - t:.1f} s to build)")
    ms_b, _ = timed_steps(lambda: batch.launch(stream), K, W, stream)
    ms_p = float("nan")
    if plain:
        batch_t = fh.Batch(plans_t, peaks, maps)  # its per-map launches (fh_batch_launch_plain)
        ms_p, _ = timed_steps(lambda: batch_t.launch_plain(stream), K, W, stream)
        batch_t.destroy()
        batch.launch(stream)  # the maps checked below are the batch's
    log(f"batched graph {ms_b:.4f} ms, plain per-map {ms_p:.4f} ms")
    # HBM roofline of the batch: algorithmic bytes = every map stored once, every
    # map's peaks, CSR and tables read once, over the graph launch's time (the
    # clearing prologue and the persistent queue kernel; HIP events on its stream)
    alg_b = sum(4 * pl.n_k * pl.n_x0 + 4 * p.n_peaks + 4 * (s.n_fft + 1) + 8 * (pl.n_f + 1) + 8 * pl.n_k + 8 * s.n_fft
                for s, p, pl in zip(specs, pms, plans))
    ach_b = alg_b / (ms_b * 1e-3) / 1e9
    roof_b = {"bound": "hbm", "achieved": round(ach_b, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
              "frac": round(ach_b / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(BATCH_TRAFFIC_PROFILE),
              "kernel": "fh::k_queue (the batch's persistent queue kernel, "
                        + (f"{plans[0].tile['threads']}-thread work-groups)"
                           if len({pl.tile["threads"] for pl in plans}) == 1 else "the library's shared work-group size)"),
              "alg_bytes": alg_b, "timing": "the whole graph launch (prologue + queue kernel), HIP events"}
    out.update({"workload": "48 uneven maps (n x T_FFT x 2 seeds, 64 Hz bands, 2 h - 3 d, 64-1024 k)",
                "tiles": "autotuned for the batch's graph launch" if tiles_b else "the library's own shapes",
                "plain": "fh_hough map by map, each with its autotuned tile shape",
                "updates_per_launch": Ub, "ms_batched": round(ms_b, 5),
                "updates_per_s_batched": Ub / (ms_b * 1e-3), "roofline": roof_b})
    if plain:
        out.update({"ms_plain": round(ms_p, 5), "updates_per_s_plain": Ub / (ms_p * 1e-3),
                    "speedup_vs_plain": round(ms_p / ms_b, 3)})
    if check_oracle:
        # every map of the batch against the oracle, and the (peak, row) pairs that
        # land in the grid (each one +1 and one -1 LDS atomic in the tile kernel)
        from oracle import hough as oracle
        t = time.perf_counter()
        pairs_b, equal_b = 0, True
        for s, p, m in zip(specs, pms, maps):
            ref_b, pr = oracle.hough(oracle.Desc.from_spec(s), p.row_ptr, p.bin, return_pairs=True)
            pairs_b += pr
            equal_b = equal_b and bool(np.array_equal(m.cpu().numpy(), ref_b))
        s_b = ms_b * 1e-3
        work_b = {"in_grid_pairs": pairs_b, "in_grid_fraction": round(pairs_b / Ub, 5),
                  "in_grid_pairs_per_s": pairs_b / s_b, "lds_atomic_lane_ops_per_s": 2 * pairs_b / s_b}
        if plain:
            work_b["in_grid_pairs_per_s_plain"] = pairs_b / (ms_p * 1e-3)
        lds_peak = 32 * 256 * 2.4e9  # LDS atomic lane-ops/s: 32 lanes/clk/CU, 256 CUs, 2.4 GHz
        work_b["lds_atomic_roof"] = {"achieved": round(2 * pairs_b / s_b / 1e12, 4), "peak": round(lds_peak / 1e12, 3),
                                     "unit": "T atomic lane-ops/s", "frac": round(2 * pairs_b / s_b / lds_peak, 4),
                                     "peak_basis": "32 lanes/clk/CU x 256 CUs x 2.4 GHz"}
        ceil_b = ceilings.load()
        if ceil_b:
            l_m = ceil_b["tests"]["lds_atomic_add_random"]["g_lane_ops_per_s"] * 1e9
            work_b["lds_atomic_frac_measured"] = round(2 * pairs_b / s_b / l_m, 4)
            work_b["lds_atomic_roof"].update(measured_peak_random=round(l_m / 1e12, 3),
                                             frac_measured=round(2 * pairs_b / s_b / l_m, 4))
        work_b["combined_roof"] = combined_roof(alg_b, pairs_b, s_b, ceil_b)
        out["work"] = work_b
        out["parity_vs_oracle"] = {"checked": f"all {len(specs)} maps", "equal": equal_b}
        log(f"batched: oracle on all maps in {time.perf_counter() - t:.1f} s, parity {equal_b}, "
            f"{pairs_b:.4e} in-grid pairs")
        assert equal_b, "batched GPU maps differ from the oracle"
    batch.destroy()
    return out


def combined_roof(alg_bytes, pairs, seconds, ceil):
    """The kernel's time against the largest of its three lower bounds (HBM on
    the algorithmic bytes, 2 LDS atomic lane-ops and 2 FP64 fma per in-grid
    pair), from the data sheet and, when stored, from the measured ceilings."""
    t = {"hbm": alg_bytes / (HBM_PEAK_GBPS * 1e9), "lds_atomic": 2.0 * pairs / (32 * 256 * 2.4e9),
         "fp64": 4.0 * pairs / (FP64_PEAK_TFLOPS * 1e12)}
    out = {"bound_us": {k: round(v * 1e6, 2) for k, v in t.items()}, "binding": max(t, key=t.get),
           "frac": round(max(t.values()) / seconds, 4)}
    if ceil:
        c = ceil["tests"]
        tm = {"hbm": alg_bytes / (c["hbm_read_1GiB"]["gb_per_s"] * 1e9),
              "lds_atomic": 2.0 * pairs / (c["lds_atomic_add_random"]["g_lane_ops_per_s"] * 1e9),
              "fp64": 4.0 * pairs / (c["fp64_fma"]["tflops"] * 1e12)}
        out.update(bound_us_measured={k: round(v * 1e6, 2) for k, v in tm.items()},
                   binding_measured=max(tm, key=tm.get), frac_measured=round(max(tm.values()) / seconds, 4))
    return out


def oracle_single_thread(n_k, n_rows=32):
    """The oracle on one host thread (a child process with OMP_NUM_THREADS=1):
    n_rows evenly spaced k rows of the large map, direct per-cell counting."""
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r)\n"
            "from paper_1810_09784_amd import synth\n"
            "from oracle import hough as oracle\n"
            "spec = synth.cfg_single_large(); pm = synth.make_peakmap(spec)\n"
            "rows = list(range(0, %d, %d))[:%d]\n"
            "t = time.perf_counter(); oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin, rows=rows)\n"
            "dt = time.perf_counter() - t\n"
            "print(json.dumps({'rows': len(rows), 's': dt, 'threads': oracle.threads(), "
            "'updates_per_s': len(rows) * pm.n_peaks / dt}))\n") % (ROOT, n_k, max(1, n_k // n_rows), n_rows)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def copy_calibration():
    """Three plain 1 GiB device copies: their FETCH_SIZE / WRITE_SIZE readings
    scale the counters of the other kernels to bytes."""
    import torch
    src = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def timed_steps(step, K, W, stream):
    import torch
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    wall0 = time.perf_counter()
    for _ in range(K):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return t0.elapsed_time(t1) / K, wall


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the generalized FrequencyHough here runs on a single MI355X; "
              "maps are independent and would shard across GPUs without any collective, which the "
              "library does not launch. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1810_09784_amd import ceilings, fh, synth, tune

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if a.cnn_only:
        print(json.dumps({"cnn": run_cnn(fh, dev, stream)}), flush=True)
        return
    if a.batched_only:
        b = run_batched(fh, synth, tune, ceilings, dev, stream, a.steps, a.warmup, False, plain=False)
        if a.copy_calibration:
            copy_calibration()
        print(json.dumps({"batched": b}), flush=True)
        return

    # ------------------------------------------------------------ inputs --
    t = time.perf_counter()
    spec = synth.cfg_single_large()
    pm = synth.make_peakmap(spec)
    log(f"peakmap: {pm.n_peaks} peaks, {spec.n_fft} FFTs x {spec.n_f} bins ({time.perf_counter() - t:.1f} s)")
    tile = tune.lookup(spec, pm.n_peaks)
    plan = fh.Plan.from_spec(spec, tile=tile)
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    hmap = torch.empty((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
    U = pm.n_peaks * plan.n_k
    log(f"plan: {plan.n_k} x {plan.n_x0} map, tile {plan.tile}, U = {U:.4e} (peak, row) pairs")

    K, W = a.steps, a.warmup
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    for e0, e1 in ev:  # materialise the events before handing them to the library
        e0.record(stream)
        e1.record(stream)
    torch.cuda.synchronize()
    cands = {}
    SQ_K, SQ_X0, MIN_DK = 5, 5, 3  # candidate selection: 5 x 5 squares, a second candidate >= 3 k rows away

    def select(m, st):
        cands["list"], cands["n"] = fh.fh_select(plan, m, SQ_K, SQ_X0, MIN_DK, stream=st, as_dicts=False)

    # (1) the unfused path, serial: fh_hough then fh_select on one stream, the host
    # waiting for each step
    def serial_step():
        fh.fh_hough(plan, rp, bn, hmap, stream)
        select(hmap, stream)

    ms_serial, _ = timed_steps(serial_step, K, W, stream)
    # the Hough transform alone (rank build + tiles), same launch configuration
    ms_hough, _ = timed_steps(lambda: fh.fh_hough(plan, rp, bn, hmap, stream), K, 2, stream)

    # (2) the unfused path pipelined over two map buffers and two streams: step k's
    # fh_hough (stream A) runs while step k-1's fh_select (stream B, after A's event
    # for that map) reads the other buffer
    sel_stream = torch.cuda.Stream()
    hmaps = [hmap, torch.empty_like(hmap)]
    done = [torch.cuda.Event(), torch.cuda.Event()]

    def unfused_pipelined(n):
        for k in range(n):
            j = k & 1
            fh.fh_hough(plan, rp, bn, hmaps[j], stream)
            done[j].record(stream)
            if k > 0:
                sel_stream.wait_event(done[1 - j])
                select(hmaps[1 - j], sel_stream)
        sel_stream.wait_event(done[(n - 1) & 1])
        select(hmaps[(n - 1) & 1], sel_stream)

    unfused_pipelined(W)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    unfused_pipelined(K)
    torch.cuda.synchronize()
    ms_unfused_pipe = (time.perf_counter() - t0) / K * 1e3

    # (3) the timed run: fh_hough_select (the selection's row pass fused into the tile
    # kernel's epilogue), two plans of the same map alternating, each on a stream of its
    # own, so that step k's selection kernels overlap step k+1's rank build and the
    # tail of one tile kernel the start of the next, and step k's square results are
    # fetched on the host while step k+1 runs.  Every step does the whole hot path on
    # its own map buffer; a plan's next step waits for its previous one on its stream.
    plans2 = [plan, fh.Plan.from_spec(spec, tile=tile)]

    def fused(n, streams, timed):
        for st in streams[1:]:
            st.wait_stream(streams[0])
        for k in range(n):
            j = k & 1
            if timed:
                fh.fh_plan_set_events(plans2[j], ev[k][0], ev[k][1])
            fh.fh_hough_select(plans2[j], rp, bn, hmaps[j], SQ_K, SQ_X0, MIN_DK, stream=streams[j % len(streams)])
            if k > 0:
                cands["list"], cands["n"] = fh.fh_select_results(plans2[1 - j], as_dicts=False)
        cands["list"], cands["n"] = fh.fh_select_results(plans2[(n - 1) & 1], as_dicts=False)
        for st in streams[1:]:
            streams[0].wait_stream(st)
        for p_ in plans2:
            fh.fh_plan_set_events(p_, None, None)

    def timed_fused(streams, timed_kernel):
        fused(W, streams, False)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        wall0 = time.perf_counter()
        fused(K, streams, timed_kernel)
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / K, (time.perf_counter() - wall0) / K * 1e3

    ms, wall_ms = timed_fused([stream, sel_stream], False)
    # The tile kernel's own time, for the roofline: the same steps on one stream,
    # with the library's events around each tile kernel.  On two streams the next
    # step's rank build shares the CUs with it and the next tile kernel queues
    # behind it, so events there would also count that wait; here no other launch
    # overlaps it.  These are the last launches of this kernel in the run.
    ms_one, _ = timed_fused([stream], True)
    kern_ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / K
    errs = fh.fh_device_errors(plans2[(K - 1) & 1])
    assert errs == 0, f"{errs} bad peaks"
    hmap = hmaps[(K - 1) & 1]  # the last step's map, checked against the oracle below
    log(f"step {ms:.4f} ms fused, two streams (host wall {wall_ms:.4f} ms), {ms_one:.4f} ms on one stream; unfused "
        f"{ms_unfused_pipe:.4f} ms pipelined, {ms_serial:.4f} ms serial; hough {ms_hough:.4f} ms, tile kernel "
        f"{kern_ms:.4f} ms, {cands['n']} candidates")

    # roofline of the tile kernel: algorithmic bytes = map store + peaks + CSR + tables, once
    map_bytes = 4 * plan.n_k * plan.n_x0
    peak_bytes = 4 * pm.n_peaks + 4 * (spec.n_fft + 1)
    table_bytes = 8 * (plan.n_f + 1) + 8 * plan.n_k + 8 * spec.n_fft
    alg_bytes = map_bytes + peak_bytes + table_bytes
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(),
            "kernel": f"fh::k_queue (persistent tile kernel with the fused selection epilogue, "
                      f"{plan.tile['threads']}-thread work-groups)",
            "kernel_ms": round(kern_ms, 5), "alg_bytes": alg_bytes,
            "timing": "HIP events around each tile kernel on its stream, the fused steps run on one stream so "
                      "that no other launch overlaps it"}
    # the same figures against what the chip delivers (csrc/ceilings.hip, stored by
    # python -m paper_1810_09784_amd.ceilings on an MI355X)
    ceil = ceilings.load()
    if ceil:
        t = ceil["tests"]
        rd = t["hbm_read_1GiB"]["gb_per_s"]
        real = roof["traffic"] / (kern_ms * 1e-3) / 1e9 if roof["traffic"] else None
        roof["measured_ceiling"] = {"hbm_read_gb_per_s": rd, "frac_alg_bytes": round(achieved / rd, 4),
                                    "real_traffic_gb_per_s": round(real, 1) if real else None,
                                    "frac_real_traffic": round(real / rd, 4) if real else None}

    out = {
        "metric": "FH Hough updates/s (exact int32), batched vs plain; CNN det-eff @ fixed FAP",
        "value": U / (ms * 1e-3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 index math, int32 counts",
        "data": "synthetic: seeded Exp(1) peakmap, threshold 2.5 local maxima, 20 power-law injections",
        "config": {"workload": "single map n=3, 200-1200 Hz, T_FFT=4 s, 43200 FFTs, 1024 k x 84000 x0",
                   "peaks": pm.n_peaks, "n_k": plan.n_k, "n_x0": plan.n_x0, "updates_per_step": U,
                   "update": "one (peak, k-row) pair, counted over all P x n_k pairs, including those whose "
                             "image misses the x0 grid (in_grid_pairs_per_s counts only the others)",
                   "tile": plan.tile, "parallelism": "1 GPU",
                   "step": "fh_hough_select: rank build, tile kernel with the selection's row pass fused "
                           "into its epilogue, split-tile selection pass, square reduction (5x5 squares, 2nd >= 3 "
                           "rows), host CR; two plans alternate on two streams, so consecutive steps overlap "
                           "on the GPU and the host finish overlaps the next step"},
        "stages_ms": {"step_one_stream": round(ms_one, 5),
                      "step_unfused_serial": round(ms_serial, 5), "step_unfused_pipelined": round(ms_unfused_pipe, 5),
                      "hough": round(ms_hough, 5), "fused_tile_kernel": round(kern_ms, 5),
                      "select_incl_host_serial": round(ms_serial - ms_hough, 5)},
        "step_unfused_serial_updates_per_s": U / (ms_serial * 1e-3),
        "hough_only_updates_per_s": U / (ms_hough * 1e-3),
        "roofline": roof,
        "machine": machine(),
    }

    # ---------------------------------------------------- batched (48 maps) --
    if not a.no_batched:
        out["batched"] = run_batched(fh, synth, tune, ceilings, dev, stream, K, W, not a.no_cpu_baseline)

    # ------------------------------------ the tile CNN on the matrix cores --
    if not a.no_sweep:
        out["cnn"] = run_cnn(fh, dev, stream)

    # ------------------------------------------- the full sweep and extras --
    if not a.no_sweep:
        out["sweep"], out["layout"] = run_sweep(fh, synth, dev, stream, cands_large=cands, spec=spec, plan=plan, rp=rp,
                                                bn=bn, K=max(3, K // 4), check_oracle=not a.no_cpu_baseline,
                                                fap_sweeps=a.fap_sweeps)

    if a.copy_calibration:
        copy_calibration()

    # ------------------------------------- the oracle on the host cores --
    if not a.no_cpu_baseline:
        from oracle import hough as oracle
        from oracle import select as oracle_select
        n_rows = plan.n_k if a.cpu_rows <= 0 else min(a.cpu_rows, plan.n_k)
        rows = list(range(0, plan.n_k, max(1, plan.n_k // n_rows)))[:n_rows]
        whole = len(rows) == plan.n_k
        d = oracle.Desc.from_spec(spec)
        t = time.perf_counter()
        ref, in_grid = oracle.hough(d, pm.row_ptr, pm.bin, rows=None if whole else rows, return_pairs=True)
        dt_h = time.perf_counter() - t
        got = hmap.cpu().numpy() if whole else hmap[rows].cpu().numpy()
        parity = bool(np.array_equal(got, ref))
        dt_s = 0.0
        if whole:  # the step's selection too, on the oracle's own map
            _, x0m, dx, _ = oracle.grid(d)
            t = time.perf_counter()
            ref_c = oracle_select.select(ref, spec.k, x0m, dx, spec.n, 5, 5, 3)
            dt_s = time.perf_counter() - t
            got_c = cands["list"]
            parity = parity and len(ref_c) == len(got_c) == cands["n"] and all(
                int(g[f]) == r[f] for g, r in zip(got_c, ref_c) for f in ("row", "col", "count", "square", "second")
            ) and all(float(g[f]) == r[f] for g, r in zip(got_c, ref_c) for f in ("cr", "mu", "sigma", "f0", "fdot0"))
        threads = oracle.threads()
        sample = (f"the whole step on the same map: direct per-cell Hough counting of all {plan.n_k} k rows x "
                  f"{pm.n_peaks} peaks ({dt_h:.2f} s, OpenMP over rows) + the 5 x 5 square selection "
                  f"({dt_s:.2f} s, numpy)") if whole else (
                  f"{len(rows)} of {plan.n_k} k rows (every {plan.n_k // len(rows)}th) of the same map, all "
                  f"{pm.n_peaks} peaks, direct per-cell counting, {dt_h:.2f} s wall; no selection")
        out["cpu_baseline"] = {"value": len(rows) * pm.n_peaks / (dt_h + dt_s), "unit": "updates/s",
                               "cores": threads, "kind": "oracle", "sample": sample,
                               "single_thread": oracle_single_thread(plan.n_k)}
        out["parity_vs_oracle"] = {"checked": "whole map and candidates" if whole else f"{len(rows)} sampled rows",
                                   "equal": parity}
        if whole:
            # the work the map really contains: (peak, row) pairs whose clipped interval
            # holds a column (counted by the oracle), each 2 FP64 fma + 2 FP64->int
            # conversions and 2 LDS atomic edge updates in the tile kernel; roofs for
            # those per-pair costs at the fused tile kernel's measured time
            s_k = roof["kernel_ms"] * 1e-3
            fp64 = 4.0 * in_grid / s_k / 1e12
            lds = 2.0 * in_grid / s_k / 1e12
            lds_peak = 32 * 256 * 2.4e9 / 1e12  # 32 lanes/clk/CU, 256 CUs, 2.4 GHz
            out["in_grid_pairs_per_step"] = in_grid
            out["cpu_baseline"]["in_grid_pairs_per_s"] = in_grid / (dt_h + dt_s)
            out["in_grid_pairs_per_s"] = in_grid / (ms * 1e-3)
            out["step_unfused_serial_in_grid_pairs_per_s"] = in_grid / (ms_serial * 1e-3)
            out["hough_only_in_grid_pairs_per_s"] = in_grid / (ms_hough * 1e-3)
            out["work"] = {"in_grid_pairs": in_grid, "in_grid_fraction": round(in_grid / U, 5),
                           "in_grid_pairs_per_s": in_grid / s_k,
                           "fp64_roof": {"achieved": round(fp64, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                         "frac": round(fp64 / FP64_PEAK_TFLOPS, 4)},
                           "lds_atomic_roof": {"achieved": round(lds, 3), "peak": round(lds_peak, 3),
                                               "unit": "T atomic lane-ops/s", "frac": round(lds / lds_peak, 4),
                                               "peak_basis": "32 lanes/clk/CU x 256 CUs x 2.4 GHz"}}
            if ceil:
                t = ceil["tests"]
                f_m = t["fp64_fma"]["tflops"]
                l_m = t["lds_atomic_add_random"]["g_lane_ops_per_s"] / 1e3
                out["work"]["fp64_roof"].update(measured_peak=f_m, frac_measured=round(fp64 / f_m, 4))
                out["work"]["lds_atomic_roof"].update(measured_peak_random=round(l_m, 3),
                                                      frac_measured=round(lds / l_m, 4))
            out["work"]["combined_roof"] = combined_roof(alg_bytes, in_grid, s_k, ceil)
        log(f"oracle: {len(rows)} rows in {dt_h:.2f} s + selection {dt_s:.2f} s on {threads} threads; "
            f"parity {parity}")
        assert parity, "GPU output differs from the oracle"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
