"""The oracle's row checker for large maps (orc_rows_checked): its early exits
must not change anything, so on small maps its rows, row totals and in-grid
pair counts equal the plain direct oracle's."""
import numpy as np
import pytest

from oracle import hough as O
from paper_1810_09784_amd import synth


def _check(d, pm, rows):
    ref = O.hough(d, pm.row_ptr, pm.bin, rows=rows)
    got, tot, prs = O.rows_checked(d, pm.row_ptr, pm.bin, rows)
    assert np.array_equal(got, ref)
    assert np.array_equal(tot, ref.astype(np.int64).sum(axis=1))
    for q, r in enumerate(rows):
        _, p = O.hough(d, pm.row_ptr, pm.bin, rows=[r], return_pairs=True)
        assert prs[q] == p
    _, tot2, prs2 = O.rows_checked(d, pm.row_ptr, pm.bin, rows, with_map=False)
    assert np.array_equal(tot2, tot) and np.array_equal(prs2, prs)
    return tot


@pytest.mark.parametrize("seed,n,kscale", [(1, 3.0, 1.0), (2, 5.0, 4.0), (3, 2.0, 20.0), (4, 7.0, 0.3)])
def test_rows_checked_equals_plain_oracle(seed, n, kscale):
    rng = np.random.default_rng(seed)
    spec = synth.cfg_tiny(rng, n_fft=300, n_f=48, n_k=24, n=n, tfft=2.0, f_min=100.0, kscale=kscale)
    pm = synth.random_peakmap(rng, spec.n_fft, spec.n_f, 0.12)
    d = O.Desc.from_spec(spec)
    tot = _check(d, pm, list(range(spec.n_k)))
    assert tot[0] > 0 and (kscale < 4.0 or tot[-1] < tot[0])  # high rows leave the grid early


def test_rows_checked_explicit_times_bad_bins_and_row_order():
    rng = np.random.default_rng(7)
    spec = synth.cfg_tiny(rng, n_fft=200, n_f=40, n_k=16, n=4.0, kscale=3.0)
    pm = synth.random_peakmap(rng, spec.n_fft, spec.n_f, 0.15)
    # bins outside the band (skipped, not an exit): one below at the front, one above at the end
    b = pm.bin.copy()
    starts = pm.row_ptr[:-1][np.diff(pm.row_ptr) > 1]
    b[starts[::3]] = -5
    ends = pm.row_ptr[1:][np.diff(pm.row_ptr) > 1] - 1
    b[ends[::4]] = spec.n_f + 3
    pm.bin = b
    t = np.cumsum(rng.uniform(0.5, 3.0, spec.n_fft))
    d = O.Desc(spec.n, spec.tfft, spec.f_min, spec.f_max, spec.n_fft, spec.k, t=t)
    _check(d, pm, [15, 0, 7, 3, 3])


def test_rows_checked_without_exits():
    rng = np.random.default_rng(9)
    spec = synth.cfg_tiny(rng, n_fft=120, n_f=32, n_k=10, n=3.0, kscale=5.0)
    pm = synth.random_peakmap(rng, spec.n_fft, spec.n_f, 0.2)
    # an FFT whose bins are not ascending switches the exits off
    i = int(np.argmax(np.diff(pm.row_ptr)))
    a, e = pm.row_ptr[i], pm.row_ptr[i + 1]
    pm.bin[a:e] = pm.bin[a:e][::-1].copy()
    _check(O.Desc.from_spec(spec), pm, list(range(spec.n_k)))
    # n = 0 (the original FrequencyHough, x = f): A grows with the bin, no exits
    d0 = O.Desc(0.0, 2.0, 100.0, 116.0, 60, np.linspace(0.0, 0.05, 6), dx0=-0.5, x0_min=116.0, n_x0=40)
    pm0 = synth.random_peakmap(rng, 60, 32, 0.2)
    _check(d0, pm0, list(range(6)))
