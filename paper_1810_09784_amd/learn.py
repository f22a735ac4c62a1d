"""The learned tile proposer: data, training and the comparison with the plain
candidate selection.

Maps.  Many small maps are needed, so their peakmaps are drawn on the GPU
(torch, seeded) with the model of synth.py: Exp(1) pixel powers, a peak is a
local maximum >= 2.5 (edge bins excluded), an injected power-law signal puts
|z + sqrt(a)|^2 (z circular complex Gaussian) into the bin holding f(t) at each
FFT mid-time.  Geometry of every map: n = 5, 500-600 Hz, T_FFT = 2 s, 7200
FFTs (4 h), 128 uniform k rows on [0, 2 k_ref) with k_ref the k of
(f0 = 580 Hz, tau = 1e4 s), 323 x0 columns -> 2 x 6 tiles of 64 x 64.
Injections: f0 ~ U(505, 595) Hz, k ~ U(0.1, 1.9) k_ref, amplitude a.

Training.  Positive tiles: the tile holding an injection's true (x0, k) cell,
a log-uniform in [0.25, 6] (weaker signals leave no trace to learn from);
negative tiles: all tiles of noise-only maps.
Rows are normalised by their map row's mean and standard deviation.

Evaluation.  A map is detected by a pipeline when one of its candidates has
CR >= its threshold and lies within 3 bins (Euclidean, in x0 and k bins) of
the injection's true cell.  Plain: the candidates of the selection over the
whole map (4 x 6 squares, second candidate 3 k rows away).  Learned: the
network scores the map's 12 tiles and the selection re-checks its top tile(s)
alone (fh_batch_select_tiles: 2 x 1 squares of 32 x 64 cells inside the 64 x
64 tile, statistics from the tile's cells), so it reads 1 of 12 tiles.  Each
pipeline's CR threshold is set on noise-only maps so that the fraction of
noise maps with a candidate above it (the false-alarm probability per map) is
the target FAP.  Maps go through the library in batches (one persistent
launch, one batched selection, one batched proposal and one batched re-check
per batch)."""
from __future__ import annotations

import math
import os
from typing import Dict, List, Tuple

import numpy as np

N_BRAKE, F_MIN, F_MAX, TFFT, N_FFT, N_K = 5.0, 500.0, 600.0, 2.0, 7200, 128
F_REF, TAU_REF = 580.0, 1e4
THETA = 2.5
SQ_K, SQ_X0 = 4, 6


def k_ref() -> float:
    return 1.0 / (TAU_REF * (N_BRAKE - 1.0) * F_REF ** (N_BRAKE - 1.0))


def k_grid() -> np.ndarray:
    return np.arange(N_K, dtype=np.float64) * ((2.0 * k_ref()) / N_K)


class MapFactory:
    """Peakmaps of the evaluation geometry, drawn on the GPU in batches."""

    def __init__(self, dev, seed: int):
        import torch
        from . import fh
        self.torch = torch
        self.dev = dev
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(int(seed))
        self.n_f = int(round((F_MAX - F_MIN) * TFFT))
        self.plan = fh.Plan(N_BRAKE, TFFT, F_MIN, F_MAX, N_FFT, k_grid())
        self.t = (torch.arange(N_FFT, dtype=torch.float64, device=dev) + 0.5) * TFFT
        self.x0_min, self.dx0 = self.plan.info.x0_min, self.plan.info.dx0

    def true_cell(self, f0: float, k: float) -> Tuple[int, int]:
        col = int(math.floor((f0 ** (1.0 - N_BRAKE) - self.x0_min) / self.dx0))
        row = int(math.floor(k / (2.0 * k_ref() / N_K) + 0.5))
        return row, col

    def draw(self, inj: List[Tuple[float, float, float]]):
        """One peakmap per entry (f0, k, a); a <= 0 means noise only.
        Returns a list of (row_ptr, bin) int32 CUDA tensors."""
        torch = self.torch
        B = len(inj)
        p = -torch.log1p(-torch.rand((B, N_FFT, self.n_f), generator=self.gen, device=self.dev))
        for b, (f0, k, a) in enumerate(inj):
            if a <= 0:
                continue
            # power law of Sec. II at the FFT mid-times
            f = f0 / (1.0 + k * (N_BRAKE - 1.0) * f0 ** (N_BRAKE - 1.0) * self.t) ** (1.0 / (N_BRAKE - 1.0))
            j = torch.floor((f - F_MIN) * TFFT)
            ok = (j >= 0) & (j < self.n_f)
            i_idx = torch.nonzero(ok).squeeze(1)
            j_idx = j[ok].long()
            g = torch.randn((2, i_idx.numel()), generator=self.gen, device=self.dev)
            re = g[0] * math.sqrt(0.5) + math.sqrt(a)
            im = g[1] * math.sqrt(0.5)
            p[b, i_idx, j_idx] = re * re + im * im
        c = p[:, :, 1:-1]
        m = (c >= THETA) & (c > p[:, :, :-2]) & (c > p[:, :, 2:])
        out = []
        for b in range(B):
            nz = torch.nonzero(m[b])
            counts = torch.bincount(nz[:, 0], minlength=N_FFT)
            rp = torch.zeros(N_FFT + 1, dtype=torch.int32, device=self.dev)
            rp[1:] = torch.cumsum(counts, 0).to(torch.int32)
            out.append((rp.contiguous(), (nz[:, 1] + 1).to(torch.int32).contiguous()))
        return out

    def hough(self, peaks):
        from . import fh
        return [fh.fh_hough(self.plan, rp, bn) for rp, bn in peaks]


def random_injection(rng: np.random.Generator, a: float):
    return float(rng.uniform(505.0, 595.0)), float(rng.uniform(0.1, 1.9) * k_ref()), float(a)


def tile_of(row: int, col: int) -> int:
    n_tb = (323 + 63) // 64
    return (row // 64) * n_tb + (col // 64)


def build_training_set(dev, n_pos: int, n_neg_maps: int, seed: int, batch: int = 32, amp_lo: float = 0.25,
                       amp_hi: float = 6.0):
    """(tiles bf16 [N, 64, 64], labels float32 [N]) on the GPU."""
    import torch
    from . import fh
    rng = np.random.default_rng(seed)
    fac = MapFactory(dev, seed + 1)
    org = torch.tensor([[64 * (t // 6), 64 * (t % 6)] for t in range(12)], dtype=torch.int32, device=dev)
    tiles, labels = [], []
    for b0 in range(0, n_pos, batch):
        inj = [random_injection(rng, math.exp(rng.uniform(math.log(amp_lo), math.log(amp_hi))))
               for _ in range(min(batch, n_pos - b0))]
        maps = fac.hough(fac.draw(inj))
        for (f0, k, a), H in zip(inj, maps):
            r, c = fac.true_cell(f0, k)
            t = tile_of(min(r, N_K - 1), min(max(c, 0), 322))
            tiles.append(fh.fh_tiles(H, org[t:t + 1].contiguous()))
            labels.append(1.0)
    for b0 in range(0, n_neg_maps, batch):
        maps = fac.hough(fac.draw([(0.0, 0.0, 0.0)] * min(batch, n_neg_maps - b0)))
        for H in maps:
            tiles.append(fh.fh_tiles(H, org))
            labels.extend([0.0] * 12)
    X = torch.cat(tiles, 0).contiguous()
    y = torch.tensor(labels, dtype=torch.float32, device=dev)
    return X, y


def train(net, X, y, epochs: int, lr: float, batch: int, seed: int, log=None, checkpoint: str = None,
          after_epoch=None) -> List[float]:
    """Adam over shuffled batches (the order drawn from `seed`); returns the mean
    loss of every epoch.  checkpoint: path of an .npz written after every epoch
    (parameters, Adam moments and step count, the epoch, the batch-order
    generator's state and the losses so far, with the run's seed, batch, lr and
    sample count); when it exists the run resumes after its epoch, and a file
    from another run (different seed, batch, lr or samples) raises ValueError.
    after_epoch(ep) is called once an epoch's checkpoint is written."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    n = X.shape[0]
    hist, start = [], 0
    run = np.array([seed, batch, n], dtype=np.int64)
    if checkpoint and os.path.exists(checkpoint):
        with np.load(checkpoint) as ck:
            if not (np.array_equal(ck["run"], run) and float(ck["lr"]) == float(lr)):
                raise ValueError(f"{checkpoint} belongs to another training run")
            net.set_params(ck["params"])
            net.set_state(ck["m1"], ck["m2"], int(ck["steps"]))
            g.set_state(torch.from_numpy(ck["rng"].copy()))
            hist = [float(v) for v in ck["hist"]]
            start = int(ck["epoch"]) + 1
        if log:
            log(f"resumed from {checkpoint} after epoch {start - 1}")
    for ep in range(start, epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            net.forward(X[idx].contiguous())
            loss = net.backward(y[idx].contiguous())
            net.step(lr)
            tot += float(loss.item())
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
        if checkpoint:
            params, _ = net.get_params()
            m1, m2, steps = net.get_state()
            tmp = checkpoint + ".tmp.npz"
            np.savez(tmp, params=params, m1=m1, m2=m2, steps=np.int64(steps), epoch=np.int64(ep),
                     rng=g.get_state().numpy(), hist=np.asarray(hist, dtype=np.float64), run=run,
                     lr=np.float64(lr))
            os.replace(tmp, checkpoint)  # a run killed while writing keeps the previous epoch's file
        if after_epoch:
            after_epoch(ep)
    return hist


TILE_SQ = (2, 1)  # squares of the re-check inside a 64 x 64 tile (32 x 64 cells, like the plain 32 x 54)


def map_statistics(fac: MapFactory, net, inj: List[Tuple[float, float, float]], n_top: int = 1):
    """Per map of one batch: (largest CR of the plain selection's candidates
    within 3 bins of the injection's true cell, or of all candidates for a
    noise map; the same for the re-check of the network's top tile(s))."""
    import torch
    from . import fh
    peaks = fac.draw(inj)
    maps = [torch.empty((fac.plan.n_k, fac.plan.n_x0), dtype=torch.int32, device=fac.dev) for _ in inj]
    b = fh.Batch([fac.plan] * len(inj), peaks, maps)
    b.launch()
    plain = b.select(SQ_K, SQ_X0, 3, as_dicts=False)
    _, tops = fh.fh_batch_propose(net, b, [n_top] * len(inj))
    req = [(i, t) for i, ts in enumerate(tops) for t in ts]
    rc, counts, _ = b.select_tiles(req, TILE_SQ[0], TILE_SQ[1], 3)
    b.destroy()
    learned, at = [[] for _ in inj], 0
    for (i, _), c in zip(req, counts):
        learned[i].append(rc[at:at + c])
        at += c
    out = []
    for q, (f0, k, a) in enumerate(inj):
        lc = np.concatenate(learned[q]) if learned[q] else plain[q][:0]
        if a > 0:
            r, c = fac.true_cell(f0, k)
            near = lambda x: np.hypot(x["row"] - r, x["col"] - c) <= 3.0
            pc, lc = plain[q][near(plain[q])], lc[near(lc)]
        else:
            pc = plain[q]
        out.append((float(pc["cr"].max()) if len(pc) else -math.inf, float(lc["cr"].max()) if len(lc) else -math.inf))
    return out


def threshold_for_fap(noise_scores: np.ndarray, fap: float) -> float:
    """Smallest threshold whose exceedance fraction on noise maps is <= fap."""
    s = np.sort(np.asarray(noise_scores))[::-1]
    k = int(math.floor(fap * len(s)))
    if k >= len(s):
        return -math.inf
    return float(np.nextafter(s[k], np.inf)) if np.isfinite(s[k]) else -math.inf


def evaluate(dev, net, amps, n_noise: int, n_per_amp: int, seed: int, fap: float, batch: int = 64, log=None):
    """Both pipelines at one false-alarm probability per map: thresholds from
    n_noise noise-only maps, then n_per_amp injected maps per amplitude.  The
    two pipelines see the same maps, so their efficiencies are compared pair by
    pair: se_diff is the standard error of eff_learned - eff_plain from the
    maps where exactly one pipeline detects (McNemar)."""
    rng = np.random.default_rng(seed)
    fac = MapFactory(dev, seed + 7)
    noise = []
    for b0 in range(0, n_noise, batch):
        noise += map_statistics(fac, net, [(0.0, 0.0, 0.0)] * min(batch, n_noise - b0))
    noise = np.array(noise)
    thr_plain = threshold_for_fap(noise[:, 0], fap)
    thr_learn = threshold_for_fap(noise[:, 1], fap)
    res: Dict[str, object] = {"fap": fap, "n_noise_maps": n_noise, "thr_plain": thr_plain, "thr_learned": thr_learn,
                              "fap_plain": float(np.mean(noise[:, 0] >= thr_plain)),
                              "fap_learned": float(np.mean(noise[:, 1] >= thr_learn)),
                              "tiles_touched_frac": 1.0 / 12.0, "curve": []}
    if log:
        log(f"{n_noise} noise maps: thresholds plain {thr_plain:.3f}, learned {thr_learn:.3f}")
    for a in amps:
        st = []
        for b0 in range(0, n_per_amp, batch):
            st += map_statistics(fac, net, [random_injection(rng, a) for _ in range(min(batch, n_per_amp - b0))])
        st = np.array(st)
        dp, dl = st[:, 0] >= thr_plain, st[:, 1] >= thr_learn
        e_p, e_l = float(np.mean(dp)), float(np.mean(dl))
        n = len(st)
        p10, p01 = float(np.mean(dp & ~dl)), float(np.mean(dl & ~dp))
        se_diff = math.sqrt(max(p10 + p01 - (p01 - p10) ** 2, 0.0) / n)
        res["curve"].append({"amp": a, "n": n, "eff_plain": e_p, "eff_learned": e_l,
                             "se_plain": math.sqrt(e_p * (1 - e_p) / n), "se_learned": math.sqrt(e_l * (1 - e_l) / n),
                             "diff": e_l - e_p, "se_diff": se_diff})
        if log:
            log(f"a = {a}: plain {e_p:.4f}, learned {e_l:.4f} (difference {e_l - e_p:+.4f} +- {se_diff:.4f})")
    return res


def build_training_set_sweep(dev, n_peakmaps: int, seed: int, inj_per_map: int = 8, t_obs: float = 5 * 86400.0,
                             n_k: int = 256, amp_lo: float = 0.5, amp_hi: float = 6.0, log=None):
    """Tiles of the full sweep's geometry (bands of 64 Hz from 100 Hz, T_FFT 2,
    4 or 8 s, n in 2..7, 5 days, 256 uniform k rows): per peakmap one (band,
    T_FFT, n) with inj_per_map sources of that n on k rows 2..127 (f0 spread over
    the band, a log-uniform in [amp_lo, amp_hi]); positives are the tiles
    holding the sources' true cells, negatives as many random tiles holding
    none.  Returns (tiles bf16 [N, 64, 64], labels float32 [N])."""
    import torch
    from . import fh, sweep
    from . import synth as S
    rng = np.random.default_rng(seed)
    bands = sweep.band_edges(30)
    tiles, labels = [], []
    for q in range(n_peakmaps):
        lo, hi = bands[int(rng.integers(len(bands)))]
        tfft = float(rng.choice(sweep.TFFTS))
        n = float(rng.choice(sweep.N_VALUES))
        n_fft = int(t_obs / tfft)
        kk = S.uniform_k((1.0 / tfft ** 2) / lo ** n, n_k)
        edges = np.linspace(lo + 3.0, hi - 3.0, inj_per_map + 1)
        injs, cells = [], []
        for e in range(inj_per_map):
            f0 = float(rng.uniform(edges[e], edges[e + 1]))
            m = int(rng.integers(2, n_k // 2))
            amp = math.exp(rng.uniform(math.log(amp_lo), math.log(amp_hi)))
            injs.append(S.Injection(f0=f0, tau=1.0 / (kk[m] * (n - 1) * f0 ** (n - 1)), n=n, amp=amp))
            cells.append((m, f0))
        spec = S.MapSpec("train", n, tfft, lo, hi, n_fft, kk, seed=seed * 1000003 + q, injections=injs)
        rp, bn, _ = S.gpu_peakmap(spec, dev)
        plan = fh.Plan.from_spec(spec)
        H = fh.fh_hough(plan, rp, bn)
        tb = (plan.n_x0 + 63) // 64
        ta = (plan.n_k + 63) // 64
        pos = set()
        for (m, f0) in cells:
            col = int(math.floor((f0 ** (1.0 - n) - plan.info.x0_min) / plan.info.dx0))
            col = min(max(col, 0), plan.n_x0 - 1)
            pos.add((m // 64) * tb + col // 64)
        neg_pool = [t for t in range(ta * tb) if t not in pos]
        negs = list(rng.choice(neg_pool, size=min(len(pos), len(neg_pool)), replace=False)) if neg_pool else []
        ids = sorted(pos) + [int(t) for t in negs]
        org = torch.tensor([[64 * (t // tb), 64 * (t % tb)] for t in ids], dtype=torch.int32, device=dev)
        tiles.append(fh.fh_tiles(H, org))
        labels += [1.0] * len(pos) + [0.0] * len(negs)
        if log and q % 100 == 0:
            log(f"training maps {q}/{n_peakmaps}")
    X = torch.cat(tiles, 0).contiguous()
    y = torch.tensor(labels, dtype=torch.float32, device=dev)
    return X, y
