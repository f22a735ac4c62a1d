"""Pins of the oracle Hough transform against what the paper and mathematics fix.

Each test targets a mistake that could plausibly sit in the oracle: the
exponent of the transform, the sign or scale of the time shift, which bin edge
is the interval's lower end, floor versus ceil, the clipping bounds, the x0 grid
step, or the accumulation loop."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1810_09784_amd import synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def power_law_f(f0, k, n, t):
    # Sec. II, Eq. powlaws: integrated frequency evolution of fdot = -k f^n
    return f0 / (1.0 + k * (n - 1.0) * f0 ** (n - 1.0) * t) ** (1.0 / (n - 1.0))


def test_transform_makes_power_law_linear(oracle):
    # Sec. IV: with x = f^(1-n), a power-law signal obeys x = x0 + (n-1) k t.
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = rng.uniform(1.5, 7.0)
        f0 = rng.uniform(100.0, 2000.0)
        tau = 10 ** rng.uniform(2, 5)
        k = 1.0 / (tau * (n - 1.0) * f0 ** (n - 1.0))  # Sec. VI.D, tau definition
        t = rng.uniform(0, 3 * tau)
        x = oracle.transform(power_law_f(f0, k, n, t), n)
        x0 = oracle.transform(f0, n)
        assert abs(x - (n - 1.0) * k * t - x0) <= 1e-11 * x
        # and x decreases with f (higher frequency -> lower x), as Sec. IV notes
        assert oracle.transform(f0 * 1.01, n) < x0


def test_x0_grid_step_is_one_bin_at_fmax(oracle):
    # Sec. VI.C: dx0 = (n-1) df / f^n at f_max, i.e. the x-width of the top bin
    # to first order in df/f_max; the grid starts at f_max^(1-n).
    for n, tfft, fmin, fmax in [(5.0, 2.0, 500.0, 600.0), (3.0, 4.0, 200.0, 1200.0), (2.5, 1.0, 100.0, 164.0),
                                (7.0, 8.0, 1000.0, 1064.0)]:
        x0min, dx0 = oracle.x0_grid(n, tfft, fmax)
        df = 1.0 / tfft
        width = (fmax - df) ** (1.0 - n) - fmax ** (1.0 - n)
        assert abs(width / dx0 - 1.0) < 2.0 * n * df / fmax
        assert x0min == pytest.approx(fmax ** (1.0 - n), rel=1e-15)
        # n_x0 covers the transformed band [f_max^(1-n), f_min^(1-n)] and no more
        nx = oracle.n_x0(n, tfft, fmin, fmax)
        span = (fmin ** (1.0 - n) - fmax ** (1.0 - n)) / dx0
        assert nx - 1 < span <= nx + 1e-6


def test_large_map_grid_is_84000_columns(oracle):
    # 200-1200 Hz, T_FFT = 4 s, n = 3: span = 1200 * (6^2 - 1) / (2 * 0.25) = 84000 exactly
    assert oracle.n_x0(3.0, 4.0, 200.0, 1200.0) == 84000
    assert oracle.n_x0(5.0, 2.0, 500.0, 600.0) == 323


def test_noiseless_injection_lands_in_one_cell(oracle):
    # A power-law signal's peaks all map to its true (x0, k) cell (Sec. IV).
    spec = S.cfg_single_small(noiseless=True)
    pm = S.make_peakmap(spec)
    n_sig = int((pm.sig_bins[0] > 0).sum() - (pm.sig_bins[0] == spec.n_f - 1).sum())
    assert pm.n_peaks == n_sig == 4017
    d = oracle.Desc.from_spec(spec)
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    inj = spec.injections[0]
    x0min, dx0 = spec.f_max ** (1 - spec.n), (spec.n - 1) * (1 / spec.tfft) / spec.f_max ** spec.n
    b_true = int(math.floor((inj.f0 ** (1 - spec.n) - x0min) / dx0))
    r_true = 64  # k grid is m * (2 k_inj / 128): k_inj is row 64 exactly
    assert spec.k[r_true] == inj.k
    assert H[r_true, b_true] == n_sig
    flat = np.sort(H.ravel())
    assert flat[-1] == n_sig and flat[-2] < n_sig  # unique maximum


@pytest.mark.parametrize("n,f0,tau,tfft,fmin,fmax,nfft", [
    (3.0, 1150.0, 3e4, 4.0, 1000.0, 1200.0, 3000),
    (2.5, 330.0, 5e3, 1.0, 300.0, 340.0, 9000),
    (7.0, 1040.0, 2e4, 2.0, 990.0, 1050.0, 4000),
])
def test_noiseless_injection_other_indices(oracle, n, f0, tau, tfft, fmin, fmax, nfft):
    inj = S.Injection(f0=f0, tau=tau, n=n, amp=5.0)
    k = np.arange(64, dtype=np.float64) * ((2.0 * inj.k) / 64.0)
    spec = S.MapSpec(name="t", n=n, tfft=tfft, f_min=fmin, f_max=fmax, n_fft=nfft, k=k, seed=0,
                     injections=[inj], noiseless=True)
    pm = S.make_peakmap(spec)
    H = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin)
    x0min, dx0 = fmax ** (1 - n), (n - 1) * (1 / tfft) / fmax ** n
    b_true = int(math.floor((f0 ** (1 - n) - x0min) / dx0))
    assert H[32, b_true] == pm.n_peaks > 100
    assert (H == pm.n_peaks).sum() >= 1 and H.max() == pm.n_peaks


def test_k0_row_is_the_bin_histogram(oracle):
    # At k = 0 no time shift applies: row 0 is each bin's peak count spread over
    # the columns its x-image (X_{j+1}, X_j] meets.
    spec = S.cfg_single_small(seed=5)
    pm = S.make_peakmap(spec)
    d = oracle.Desc.from_spec(spec)
    H0 = oracle.hough(d, pm.row_ptr, pm.bin, rows=[0])[0]
    A, _, _ = oracle.tables(d)
    nf, x0min, dx0, nx = oracle.grid(d)
    # the table itself against an independent evaluation of the transform
    fj = spec.f_min + np.arange(nf + 1) / spec.tfft
    A_np = (fj ** (1 - spec.n) - spec.f_max ** (1 - spec.n)) / dx0
    np.testing.assert_allclose(A, A_np, rtol=1e-12, atol=1e-9)
    assert A[nf] == 0.0 and np.all(np.diff(A) < 0)
    cnt = np.bincount(pm.bin, minlength=nf)
    ref = np.zeros(nx, dtype=np.int64)
    for j in range(nf):
        lo, hi = int(math.floor(A[j + 1])), min(int(math.floor(A[j])), nx - 1)
        ref[max(lo, 0):hi + 1] += cnt[j]
    np.testing.assert_array_equal(H0, ref)


def _exact_map(A, Cr, T, row_ptr, bins, nx):
    """Exact-rational Hough map of tiny maps: peak (i, j) at row r meets column b
    iff the half-open image (A[j+1] - C_r T_i, A[j] - C_r T_i] meets [b, b+1)."""
    nk = len(Cr)
    H = np.zeros((nk, nx), dtype=np.int64)
    near = 0
    Af = [Fraction(a) for a in A]
    for r in range(nk):
        c = Fraction(Cr[r])
        for i in range(len(row_ptr) - 1):
            s = c * Fraction(T[i])
            for p in range(row_ptr[i], row_ptr[i + 1]):
                j = int(bins[p])
                lo, hi = Af[j + 1] - s, Af[j] - s
                for u in (lo, hi):  # an inexact edge within 2 ulp of an integer may round onto it
                    if 0 < abs(u - round(u)) <= 2 * abs(float(u)) * 2.0 ** -52:
                        near += 1
                for b in range(nx):
                    if lo < b + 1 and hi >= b:
                        H[r, b] += 1
    return H, near


@pytest.mark.parametrize("seed", range(6))
def test_exact_rational_bruteforce(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    n = float(rng.choice([2.0, 2.5, 3.0, 5.0, 7.0]))
    tfft = float(rng.choice([1.0, 2.0, 4.0]))
    nf = int(rng.integers(3, 17))
    fmin = float(rng.integers(50, 400))
    spec = S.cfg_tiny(rng, n_fft=int(rng.integers(1, 17)), n_f=nf, n_k=int(rng.integers(1, 9)), n=n, tfft=tfft,
                      f_min=fmin, kscale=float(rng.choice([1e-4, 1e-3, 1e-2])))
    pm = S.random_peakmap(rng, spec.n_fft, nf, 0.3)
    d = oracle.Desc.from_spec(spec)
    nf_, x0min, dx0, nx = oracle.grid(d)
    if seed % 2:  # a truncated grid: the right-hand clip must hold
        d = oracle.Desc.from_spec(spec, n_x0=max(1, nx // 2))
        nx = max(1, nx // 2)
    assert nx <= 400
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    A, Cr, T = oracle.tables(d)
    E, near = _exact_map(A, Cr, T, pm.row_ptr, pm.bin, nx)
    assert near == 0  # none occur for these seeds; the comparison below is exact
    np.testing.assert_array_equal(H, E)


@pytest.mark.parametrize("seed", range(4))
def test_n0_reduces_to_original_frequency_hough(oracle, seed):
    # Sec. III: the original FH maps a peak (t, f) to the line f0 = f - fdot t.
    # With n = 0 the generalized transform is x = f and k = -fdot, so the
    # oracle's map must equal an exact count of f0-cells met by
    # [f_j + k t, f_{j+1} + k t), the f0 cells being (f_max-(b+1)df, f_max-b df].
    rng = np.random.default_rng(200 + seed)
    tfft = float(rng.choice([1.0, 2.0, 4.0]))
    nf = int(rng.integers(4, 20))
    fmin = float(rng.integers(50, 500))
    fmax = fmin + nf / tfft
    nfft = int(rng.integers(2, 12))
    k = np.sort(rng.uniform(1e-5, 2e-3, int(rng.integers(1, 6))))
    pm = S.random_peakmap(rng, nfft, nf, 0.35)
    d = oracle.Desc(0.0, tfft, fmin, fmax, nfft, k)
    nf_, x0min, dx0, nx = oracle.grid(d)
    assert nx == nf and x0min == fmax and dx0 == -1.0 / tfft
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    df = Fraction(1) / Fraction(tfft)
    E = np.zeros_like(H)
    for r, kr in enumerate(k):
        kq = Fraction(kr)
        for i in range(nfft):
            t = (Fraction(i) + Fraction(1, 2)) * Fraction(tfft)
            for p in range(pm.row_ptr[i], pm.row_ptr[i + 1]):
                j = int(pm.bin[p])
                a = Fraction(fmin) + j * df + kq * t
                b_ = a + df
                for b in range(nx):
                    lo_c, hi_c = Fraction(fmax) - (b + 1) * df, Fraction(fmax) - b * df
                    if a <= hi_c and b_ > lo_c:
                        E[r, b] += 1
    np.testing.assert_array_equal(H, E)


def test_additive_and_order_free(oracle):
    rng = np.random.default_rng(7)
    spec = S.cfg_tiny(rng, n_fft=300, n_f=120, n_k=24, n=4.0, tfft=2.0, f_min=300.0, kscale=0.05)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.1)
    d = oracle.Desc.from_spec(spec)
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    # split every FFT's peaks into two random halves
    keep = rng.random(pm.n_peaks) < 0.5
    fft_of = np.repeat(np.arange(spec.n_fft), np.diff(pm.row_ptr))

    def sub(mask):
        rp = np.zeros(spec.n_fft + 1, dtype=np.int32)
        rp[1:] = np.cumsum(np.bincount(fft_of[mask], minlength=spec.n_fft))
        return rp, pm.bin[mask]

    H1 = oracle.hough(d, *sub(keep))
    H2 = oracle.hough(d, *sub(~keep))
    np.testing.assert_array_equal(H, H1 + H2)
    # reverse the peak order inside every FFT
    b2 = pm.bin.copy()
    for i in range(spec.n_fft):
        b2[pm.row_ptr[i]:pm.row_ptr[i + 1]] = b2[pm.row_ptr[i]:pm.row_ptr[i + 1]][::-1]
    np.testing.assert_array_equal(H, oracle.hough(d, pm.row_ptr, b2))


def test_row_totals_equal_interval_widths(oracle):
    rng = np.random.default_rng(8)
    spec = S.cfg_tiny(rng, n_fft=40, n_f=60, n_k=6, n=5.0, tfft=2.0, f_min=500.0, kscale=0.02)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.15)
    d = oracle.Desc.from_spec(spec)
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    fi, fj = pm.pairs()
    for r in range(spec.n_k):
        tot = sum(oracle.pair_interval(d, r, int(i), int(j))[2] for i, j in zip(fi, fj))
        assert H[r].sum() == tot


def test_in_grid_pair_count(oracle):
    # The count of (row, peak) pairs whose clipped interval holds a column:
    # at k = 0 every valid peak's image lies inside the x0 grid (the grid spans
    # the band), so row 0 counts every peak; a row whose shift moves every image
    # past x0_min counts none; any row equals the count of non-empty intervals
    # of the exact-rational brute force on a tiny map.
    rng = np.random.default_rng(12)
    spec = S.cfg_tiny(rng, n_fft=12, n_f=14, n_k=5, n=3.0, tfft=2.0, f_min=300.0, kscale=0.5)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.3)
    d = oracle.Desc.from_spec(spec)
    H, pairs = oracle.hough(d, pm.row_ptr, pm.bin, rows=[0], return_pairs=True)
    assert pairs == pm.n_peaks
    A, Cr, T = oracle.tables(d)
    nf, x0min, dx0, nx = oracle.grid(d)
    big = np.array([1e9 * (A[0] + nx) / (Cr[1] * T[0]) * spec.k[1]])  # shift > A[0] + n_x0 columns at t_0
    d_big = oracle.Desc(spec.n, spec.tfft, spec.f_min, spec.f_max, spec.n_fft, big)
    assert oracle.hough(d_big, pm.row_ptr, pm.bin, return_pairs=True)[1] == 0
    _, total = oracle.hough(d, pm.row_ptr, pm.bin, return_pairs=True)
    Af = [Fraction(a) for a in A]
    want = 0
    for r in range(spec.n_k):
        for i in range(spec.n_fft):
            s = Fraction(Cr[r]) * Fraction(T[i])
            for p in range(pm.row_ptr[i], pm.row_ptr[i + 1]):
                j = int(pm.bin[p])
                lo, hi = Af[j + 1] - s, Af[j] - s
                want += any(lo < b + 1 and hi >= b for b in range(nx))
    assert total == want


def test_bad_bins_are_skipped_and_counted(oracle):
    rng = np.random.default_rng(9)
    spec = S.cfg_tiny(rng, n_fft=10, n_f=30, n_k=4)
    pm = S.random_peakmap(rng, 10, 30, 0.2)
    d = oracle.Desc.from_spec(spec)
    H = oracle.hough(d, pm.row_ptr, pm.bin)
    b2 = pm.bin.copy()
    b2[0], b2[-1] = -1, 30
    H2, bad = oracle.hough(d, pm.row_ptr, b2, return_bad=True)
    assert bad == 2
    fi, fj = pm.pairs()
    for q in (0, pm.n_peaks - 1):
        one = np.zeros(11, dtype=np.int32)
        one[fi[q] + 1:] = 1
        H -= oracle.hough(d, one, np.array([fj[q]], dtype=np.int32))
    np.testing.assert_array_equal(H, H2)


def test_peak_density_matches_p0():
    # A bin is a peak iff power >= theta and it beats both Exp(1) neighbours:
    # p0 = int_theta^inf e^-x (1 - e^-x)^2 dx = e^-t - e^-2t + e^-3t / 3.
    th = S.THETA
    p0 = math.exp(-th) - math.exp(-2 * th) + math.exp(-3 * th) / 3
    assert abs(p0 - 0.075531) < 1e-6
    spec = S.MapSpec(name="noise", n=3.0, tfft=2.0, f_min=100.0, f_max=300.0, n_fft=3000,
                     k=np.zeros(1), seed=31)
    pm = S.make_peakmap(spec)
    m = spec.n_fft * (spec.n_f - 2)
    z = (pm.n_peaks - p0 * m) / math.sqrt(m * p0 * (1 - p0))
    assert abs(z) < 5
    assert pm.bin.min() >= 1 and pm.bin.max() <= spec.n_f - 2


def test_noise_mean_per_cell(oracle):
    # E[H[r][b]] = p0 * (number of interior (FFT, bin) pairs covering (r, b)),
    # the coverage being the Hough map of a peakmap with every interior bin set.
    th = S.THETA
    p0 = math.exp(-th) - math.exp(-2 * th) + math.exp(-3 * th) / 3
    base = S.cfg_tiny(np.random.default_rng(3), n_fft=400, n_f=80, n_k=4, n=5.0, tfft=2.0, f_min=500.0,
                      kscale=0.01)
    d = oracle.Desc.from_spec(base)
    full = S.full_peakmap(base.n_fft, base.n_f)
    cov = oracle.hough(d, full.row_ptr, full.bin).astype(np.float64)
    acc = np.zeros_like(cov)
    nseed = 12
    for s in range(nseed):
        spec = S.MapSpec(**{**base.__dict__, "seed": 1000 + s})
        pm = S.make_peakmap(spec)
        acc += oracle.hough(d, pm.row_ptr, pm.bin)
    mean = acc / nseed
    sd = np.sqrt(np.maximum(cov, 1) * p0 * (1 - p0) / nseed)
    z = (mean - p0 * cov) / sd
    assert np.abs(z).max() < 6.0
    assert abs(z.mean()) < 0.2


def test_paper_figure_caption_timescale(oracle):
    # Fig. pm caption prints f0, fdot0, n and the (x0, k) of the injection; the
    # pair is internally inconsistent by a common factor (~0.45), but its ratio
    # x0 / ((n-1) k) is the spin-down timescale tau = f0 / (|fdot0| (n-1)) of
    # Sec. VI.D, which the oracle's transform must reproduce.
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)["fig_pm_caption"]
    n, f0, fd = g["n"], g["f0"], abs(g["fdot0"])
    k = fd / f0 ** n  # Sec. II, k = |fdot0| / f0^n
    tau_oracle = oracle.transform(f0, n) / ((n - 1) * k)
    assert tau_oracle == pytest.approx(f0 / (fd * (n - 1)), rel=1e-12)
    assert tau_oracle == pytest.approx(g["x0"] / ((n - 1) * g["k"]), rel=g["rel_tol_ratio"])
