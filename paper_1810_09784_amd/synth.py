"""Seeded synthetic peakmaps and workload descriptions.

This module is the only thing the oracle side and the GPU side share: it draws
the inputs (peakmaps, injected signals, k grids) and holds none of the Hough
arithmetic.

Peakmap model (Sec. III): the normalised power of each FFT bin of whitened
Gaussian noise is Exp(1); a bin is a peak when its power is at least the
threshold theta and strictly larger than both neighbours in frequency.  The
first and last bins of the band have only one neighbour and are never peaks.
A peak at bin j stands for the whole bin [f_min + j df, f_min + (j+1) df).

Signals follow the power law of Sec. II (Eq. powlaws) with the spin-down
timescale tau of Sec. VI.D:
    f(t) = f0 (1 + t/tau)^(1/(1-n)),   k = 1 / (tau (n-1) f0^(n-1)),
evaluated at the mid-time of each FFT.  A signal adds power to the one bin
that holds f(t): the bin's power becomes |z + sqrt(a)|^2 with z circular
complex Gaussian of unit variance (a non-central chi-square, mean 1 + a).

Peaks are returned as a CSR by FFT (time-major): FFT i owns
bin[row_ptr[i]:row_ptr[i+1]], ascending.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

THETA = 2.5


@dataclasses.dataclass
class Injection:
    f0: float          # frequency at t0 (Hz)
    tau: float         # spin-down timescale (s)
    n: float           # braking index of the signal
    amp: float         # added mean power a

    @property
    def k(self) -> float:
        return 1.0 / (self.tau * (self.n - 1.0) * self.f0 ** (self.n - 1.0))

    def freq(self, t: np.ndarray) -> np.ndarray:
        return self.f0 * (1.0 + t / self.tau) ** (1.0 / (1.0 - self.n))


@dataclasses.dataclass
class MapSpec:
    """One Hough map: the search parameters plus how to draw its peakmap."""
    name: str
    n: float
    tfft: float
    f_min: float
    f_max: float
    n_fft: int
    k: np.ndarray                      # float64 [n_k], ascending
    seed: int
    injections: List[Injection] = dataclasses.field(default_factory=list)
    theta: float = THETA
    noiseless: bool = False            # pixels are 0 except injected ones (= amp)

    @property
    def n_f(self) -> int:
        w = (self.f_max - self.f_min) * self.tfft
        r = int(round(w))
        assert abs(w - r) <= 1e-9 and r >= 1
        return r

    @property
    def n_k(self) -> int:
        return int(self.k.shape[0])

    def times(self) -> np.ndarray:
        return (np.arange(self.n_fft, dtype=np.float64) + 0.5) * self.tfft


@dataclasses.dataclass
class Peakmap:
    row_ptr: np.ndarray    # int32 [n_fft + 1]
    bin: np.ndarray        # int32 [n_peaks]
    n_fft: int
    n_f: int
    sig_bins: Optional[np.ndarray] = None  # int32 [n_inj, n_fft], -1 where out of band

    @property
    def n_peaks(self) -> int:
        return int(self.bin.shape[0])

    def pairs(self):
        """(fft index, bin) of every peak, as two int arrays."""
        i = np.repeat(np.arange(self.n_fft, dtype=np.int32), np.diff(self.row_ptr))
        return i, self.bin


def signal_bins(spec: MapSpec) -> np.ndarray:
    """Bin index of every injection at every FFT mid-time; -1 if out of band."""
    t = spec.times()
    df = 1.0 / spec.tfft
    out = np.full((len(spec.injections), spec.n_fft), -1, dtype=np.int32)
    for q, inj in enumerate(spec.injections):
        f = inj.freq(t)
        j = np.floor((f - spec.f_min) / df)
        ok = (j >= 0) & (j < spec.n_f)
        out[q, ok] = j[ok].astype(np.int32)
    return out


def _local_max_peaks(p: np.ndarray, theta: float):
    """Peaks of a block of FFT rows p [rows, n_f]: (row, bin) of every bin with
    power >= theta that beats both neighbours; edge bins never qualify."""
    c = p[:, 1:-1]
    m = (c >= theta) & (c > p[:, :-2]) & (c > p[:, 2:])
    r, j = np.nonzero(m)
    return r, j + 1


def make_peakmap(spec: MapSpec, chunk_rows: int = 2048) -> Peakmap:
    """Draw the peakmap of a map spec.  Deterministic in spec.seed."""
    n_f, n_fft = spec.n_f, spec.n_fft
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    sig = signal_bins(spec)
    counts = np.zeros(n_fft, dtype=np.int64)
    bins: List[np.ndarray] = []
    for i0 in range(0, n_fft, chunk_rows):
        i1 = min(n_fft, i0 + chunk_rows)
        rows = i1 - i0
        if spec.noiseless:
            p = np.zeros((rows, n_f), dtype=np.float64)
        else:
            p = rng.standard_exponential((rows, n_f))
        for q, inj in enumerate(spec.injections):
            jj = sig[q, i0:i1]
            ok = np.nonzero(jj >= 0)[0]
            if ok.size == 0:
                continue
            if spec.noiseless:
                p[ok, jj[ok]] = inj.amp
            else:
                g = rng.standard_normal((2, ok.size))
                re = g[0] * math.sqrt(0.5) + math.sqrt(inj.amp)
                im = g[1] * math.sqrt(0.5)
                p[ok, jj[ok]] = re * re + im * im
        r, j = _local_max_peaks(p, spec.theta)
        counts[i0:i1] = np.bincount(r, minlength=rows)
        bins.append(j.astype(np.int32))
    row_ptr = np.zeros(n_fft + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    b = np.concatenate(bins) if bins else np.zeros(0, dtype=np.int32)
    return Peakmap(row_ptr=row_ptr.astype(np.int32), bin=np.ascontiguousarray(b, dtype=np.int32),
                   n_fft=n_fft, n_f=n_f, sig_bins=sig)


def gpu_peakmap(spec: MapSpec, dev, chunk_rows: int = 16384):
    """The same peakmap model drawn on the GPU (torch, seeded by spec.seed; a
    different random stream from make_peakmap): (row_ptr, bin) int32 tensors
    on `dev` and the host copy of the signal bins.  For workloads too large to
    draw on the host (the full sweep)."""
    import torch
    n_f, n_fft = spec.n_f, spec.n_fft
    g = torch.Generator(device=dev)
    g.manual_seed(int(spec.seed))
    sig = signal_bins(spec)
    sig_t = torch.from_numpy(sig).to(dev) if sig.size else None
    counts, bins = [], []
    for i0 in range(0, n_fft, chunk_rows):
        i1 = min(n_fft, i0 + chunk_rows)
        rows = i1 - i0
        if spec.noiseless:
            p = torch.zeros((rows, n_f), dtype=torch.float32, device=dev)
        else:
            p = -torch.log1p(-torch.rand((rows, n_f), generator=g, device=dev))
        for q, inj in enumerate(spec.injections):
            jj = sig_t[q, i0:i1]
            ok = torch.nonzero(jj >= 0).squeeze(1)
            if ok.numel() == 0:
                continue
            if spec.noiseless:
                p[ok, jj[ok].long()] = inj.amp
            else:
                z = torch.randn((2, ok.numel()), generator=g, device=dev)
                re = z[0] * math.sqrt(0.5) + math.sqrt(inj.amp)
                im = z[1] * math.sqrt(0.5)
                p[ok, jj[ok].long()] = re * re + im * im
        c = p[:, 1:-1]
        m = (c >= spec.theta) & (c > p[:, :-2]) & (c > p[:, 2:])
        nz = torch.nonzero(m)
        counts.append(torch.bincount(nz[:, 0], minlength=rows))
        bins.append((nz[:, 1] + 1).to(torch.int32))
    cnt = torch.cat(counts)
    row_ptr = torch.zeros(n_fft + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(cnt, 0)
    assert int(row_ptr[-1].item()) < 2 ** 31
    return row_ptr.to(torch.int32).contiguous(), torch.cat(bins).contiguous(), sig


def full_peakmap(n_fft: int, n_f: int) -> Peakmap:
    """Every interior bin of every FFT is a peak (coverage counting)."""
    per = np.arange(1, n_f - 1, dtype=np.int32)
    b = np.tile(per, n_fft)
    row_ptr = (np.arange(n_fft + 1, dtype=np.int64) * per.size).astype(np.int32)
    return Peakmap(row_ptr=row_ptr, bin=b, n_fft=n_fft, n_f=n_f)


def random_peakmap(rng: np.random.Generator, n_fft: int, n_f: int, density: float) -> Peakmap:
    """Unstructured peaks (any bin, including the edge bins): for shape tests."""
    m = rng.random((n_fft, n_f)) < density
    r, j = np.nonzero(m)
    counts = np.bincount(r, minlength=n_fft)
    row_ptr = np.zeros(n_fft + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Peakmap(row_ptr=row_ptr.astype(np.int32), bin=j.astype(np.int32), n_fft=n_fft, n_f=n_f)


# ------------------------------------------------------------- workloads --

def k_max_paper(tfft: float, f_min: float, n: float) -> float:
    """Largest k of a search: the spin-down a T_FFT can follow, 1/T_FFT^2
    (Sec. VI.D, Eq. dot_tfft), at the lowest frequency (Sec. VI.B)."""
    return (1.0 / (tfft * tfft)) / f_min ** n


def uniform_k(k_max: float, n_k: int, inclusive: bool = True) -> np.ndarray:
    m = np.arange(n_k, dtype=np.float64)
    return m * (k_max / (n_k - 1)) if inclusive else m * (k_max / n_k)


def cfg_single_small(noiseless: bool = False, seed: int = 1) -> MapSpec:
    """Single map, n = 5: band 500-600 Hz, T_FFT = 2 s, 7200 FFTs (4 h); one
    injection f0 = 580 Hz, tau = 1e4 s, +8 mean power; 128 uniform k in
    [0, 2 k_inj) so that k_inj is exactly row 64."""
    inj = Injection(f0=580.0, tau=1e4, n=5.0, amp=8.0)
    k = np.arange(128, dtype=np.float64) * ((2.0 * inj.k) / 128.0)
    return MapSpec(name="single_n5_500-600Hz_T2_7200fft", n=5.0, tfft=2.0, f_min=500.0, f_max=600.0,
                   n_fft=7200, k=k, seed=seed, injections=[inj], noiseless=noiseless)


def _draw_injections(rng, n_inj, n, f_lo, f_hi, k_max, amp_lo, amp_hi, tau_lo=1e3, tau_hi=1e5):
    """f0 uniform in the band, tau log-uniform in [tau_lo, tau_hi], restricted
    to k <= k_max (the searched k range): where the whole tau range would give
    k > k_max the range is moved up to start at the smallest admissible tau."""
    out = []
    for _ in range(n_inj):
        f0 = rng.uniform(f_lo, f_hi)
        tau_min = 1.0 / (k_max * (n - 1.0) * f0 ** (n - 1.0)) * (1.0 + 1e-9)
        lo = max(tau_lo, tau_min)
        hi = max(tau_hi, 10.0 * lo)
        tau = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi))
        amp = rng.uniform(amp_lo, amp_hi)
        out.append(Injection(f0=f0, tau=tau, n=n, amp=amp))
    return out


def cfg_single_large(seed: int = 2, n_fft: int = 43200, n_k: int = 1024) -> MapSpec:
    """Large single map, n = 3: band 200-1200 Hz, T_FFT = 4 s (4000 bins),
    43200 FFTs (2 days), 20 injections (tau 1e3-1e5 s, +2..6 power), 1024 k
    values uniform on [0, k_max] with k_max from the 1/T_FFT^2 spin-down at
    f_min."""
    n, tfft, f_min, f_max = 3.0, 4.0, 200.0, 1200.0
    kmax = k_max_paper(tfft, f_min, n)
    rng = np.random.Generator(np.random.PCG64(10_000 + seed))
    inj = _draw_injections(rng, 20, n, f_min, f_max, kmax, 2.0, 6.0)
    return MapSpec(name="single_n3_200-1200Hz_T4_43200fft", n=n, tfft=tfft, f_min=f_min, f_max=f_max,
                   n_fft=n_fft, k=uniform_k(kmax, n_k), seed=seed, injections=inj)


def cfg_batched(seeds: Sequence[int] = (3, 4)) -> List[MapSpec]:
    """48 uneven maps: n in {2,2.5,3,4,5,7} x T_FFT in {1,2,4,8} s, once per
    seed; 64 Hz bands at random centres in 100-2000 Hz, durations 2 h - 3 days,
    64-1024 k rows, 0-3 injections each."""
    specs = []
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(20_000 + seed))
        for n in (2.0, 2.5, 3.0, 4.0, 5.0, 7.0):
            for tfft in (1.0, 2.0, 4.0, 8.0):
                f_min = float(rng.integers(100, 1937))
                f_max = f_min + 64.0
                t_obs = rng.uniform(7200.0, 259200.0)
                n_fft = max(1, int(t_obs // tfft))
                n_k = int(math.floor(2.0 ** rng.uniform(6.0, 10.0)))
                kmax = k_max_paper(tfft, f_min, n)
                n_inj = int(rng.integers(0, 4))
                inj = _draw_injections(rng, n_inj, n, f_min, f_max, kmax, 2.0, 6.0)
                mseed = int(rng.integers(0, 2**31 - 1))
                specs.append(MapSpec(name=f"b{seed}_n{n}_T{int(tfft)}_{int(f_min)}Hz", n=n, tfft=tfft,
                                     f_min=f_min, f_max=f_max, n_fft=n_fft, k=uniform_k(kmax, n_k),
                                     seed=mseed, injections=inj))
    return specs


def cfg_tiny(rng: np.random.Generator, n_fft: int, n_f: int, n_k: int, n: float = 3.0,
             tfft: float = 2.0, f_min: float = 100.0, kscale: float = 1.0) -> MapSpec:
    """Small random map for shape and edge tests."""
    f_max = f_min + n_f / tfft
    kmax = k_max_paper(tfft, f_min, n) * kscale
    k = np.sort(rng.uniform(0.0, kmax, n_k))
    k[0] = 0.0
    return MapSpec(name=f"tiny_{n_fft}x{n_f}x{n_k}", n=n, tfft=tfft, f_min=f_min, f_max=f_max,
                   n_fft=n_fft, k=k, seed=int(rng.integers(0, 2**31 - 1)))
