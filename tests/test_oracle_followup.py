"""Pins of the oracle follow-up (Sec. V on peakmaps)."""
import math

import numpy as np
import pytest

from oracle import followup as OF
from paper_1810_09784_amd import synth as S


def test_zero_spindown_projection_is_the_frequency_histogram():
    # k = 0: no drift, the projection is the plain count of peaks per bin
    rng = np.random.default_rng(3)
    pm = S.random_peakmap(rng, 300, 80, 0.1)
    T = (np.arange(300) + 0.5) * 2.0
    hist, _ = OF.project(pm.row_ptr, pm.bin, T, 4.0, 2.0, 100.0, 80, 120.25, 0.0, 10, 2)
    b0 = math.floor((120.25 - 100.0) * 2.0)
    plain = np.bincount(pm.bin, minlength=80)
    assert hist == [int(plain[b]) if 0 <= b < 80 else 0 for b in range(b0 - 10, b0 + 11)]


def test_noiseless_track_gathers_in_one_bin():
    # a noiseless power-law track: after the drift correction every in-band signal peak
    # sits in the candidate's initial bin
    inj = S.Injection(f0=585.3, tau=2e4, n=5.0, amp=8.0)
    spec = S.MapSpec("nl", 5.0, 2.0, 500.0, 600.0, 3000, np.array([inj.k]), seed=1, injections=[inj], noiseless=True)
    pm = S.make_peakmap(spec)
    inband = int(np.sum((pm.sig_bins[0] >= 1) & (pm.sig_bins[0] <= spec.n_f - 2)))  # edge bins are never peaks
    hist, r = OF.project(pm.row_ptr, pm.bin, spec.times(), 5.0, 2.0, 500.0, spec.n_f, inj.f0, inj.k, 30, 2)
    assert r["y"] == inband == pm.n_peaks and sum(hist) == inband


def test_critical_ratio_of_a_two_level_background():
    # noise bins alternate m and m + 2: mu = m + 1, sigma = 1, so CR = y - m - 1
    w, guard = 6, 1
    hist = [0] * (2 * w + 1)
    noise = [x for x in range(2 * w + 1) if not w - guard <= x <= w + guard]
    for i, x in enumerate(noise):
        hist[x] = 10 + 2 * (i % 2)
    hist[w] = 25
    # realise the histogram as a peakmap with k = 0 (no drift): bin b0 + d holds hist[d + w] peaks
    b0, n_f = 20, 60
    bins = sorted(b0 - w + x for x, y in enumerate(hist) for _ in range(y))
    row_ptr = np.array([0] + [len(bins)], dtype=np.int32)  # one FFT holding every peak
    _, r = OF.project(row_ptr, np.array(bins), [1.0], 3.0, 1.0, 100.0, n_f, 100.0 + b0 + 0.5, 0.0, w, guard)
    assert (r["mu"], r["sigma"], r["cr"]) == (11.0, 1.0, 25 - 11.0)


def test_roi_grid_tiles_the_coincidence_window():
    x0_min, dxf, n_x0, ks = OF.roi_grid(1.0, 5.0, 0.01, 0.5, over=10, half=3)
    assert n_x0 == 60 and dxf == pytest.approx(0.001)
    assert x0_min == pytest.approx(0.97) and x0_min + n_x0 * dxf == pytest.approx(1.03)
    assert len(ks) == 60 and ks[30] == 5.0 and np.allclose(np.diff(ks), 0.05)
    # rows below k = 0 are dropped
    assert min(OF.roi_grid(1.0, 0.5, 0.01, 0.5)[3]) >= 0 and len(OF.roi_grid(1.0, 0.5, 0.01, 0.5)[3]) == 40
