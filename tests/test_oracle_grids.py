"""Pins of the oracle's search grids (Sec. VI) against what the paper's
equations fix, by routes other than the grid code itself."""
import math

import numpy as np
import pytest

from oracle import grids as G


@pytest.mark.parametrize("n,tfft,band", [(3.0, 4.0, (200.0, 1200.0)), (5.0, 2.0, (500.0, 600.0)),
                                         (7.0, 8.0, (350.0, 800.0))])
def test_k_grid_keeps_the_spindown_at_f_max(n, tfft, band):
    # Sec. VI.B: moving f by one bin and k by dk leaves -k f^n unchanged at f_max
    f_min, f_max = band
    fd_max = 1.0 / tfft ** 2
    ks, dks = G.k_grid(n, tfft, f_min, f_max, fd_max * 1e-2, fd_max)
    df = 1.0 / tfft
    for lo, hi in zip(ks[:-1], ks[1:]):
        assert lo * (f_max + df) ** n == pytest.approx(hi * f_max ** n, rel=1e-12)
    # the Taylor form dk ~ -n k df / f_max holds to second order
    for k, dk in zip(ks, dks):
        assert dk == pytest.approx(n * k * df / f_max, rel=(n + 1) * df / f_max)
    # end points: k_max = fdot_max / f_min^n exactly, and the grid just passes k_min
    assert ks[-1] == fd_max / f_min ** n
    k_min = fd_max * 1e-2 / f_max ** n
    assert ks[0] <= k_min < ks[1]
    # number of points from the closed form of a geometric sequence
    q = (f_max / (f_max + df)) ** n
    assert len(ks) == math.ceil(math.log(k_min / ks[-1]) / math.log(q)) + 1


def test_k_grid_rejects_zero_minimum_spindown():
    with pytest.raises(ValueError):
        G.k_grid(3.0, 4.0, 200.0, 1200.0, 0.0, 1.0 / 16)


def _deviation_dense(n1, n2, f0, k, t_obs):
    # independent evaluation: the closed form on a different, denser time axis
    t = np.linspace(0.0, t_obs, 20001)
    f = lambda n: f0 * np.exp(-np.log1p(k * (n - 1) * f0 ** (n - 1) * t) / (n - 1))
    return float(np.max(np.abs(f(n2) - f(n1))))


@pytest.mark.parametrize("n", [2.5, 4.0, 6.5])
def test_n_step_confines_the_track_to_one_bin(n):
    # Sec. VI.A: at dn the power laws for n and n + dn stay within one bin over T_obs,
    # and a step 1% larger leaves it
    tfft, f0, t_obs = 2.0, 2000.0, 1e5
    fd0 = 1.0 / tfft ** 2
    dn = G.n_step(n, tfft, f0, fd0, t_obs)
    k = fd0 / f0 ** n
    assert _deviation_dense(n, n + dn, f0, k, t_obs) <= (1.0 / tfft) * (1 + 1e-3)
    assert _deviation_dense(n, n + 1.01 * dn, f0, k, t_obs) > 1.0 / tfft


def test_n_grid_thins_out_at_high_braking_index_and_long_ffts():
    # Figs. npts and n_vs_tfft: the step grows with n, and at long T_FFT (small spindowns,
    # Taylor regime) it is larger than at T_FFT = 2 s
    grid = G.n_grid(2.5, 2.502, 2.0, 2000.0, 0.25, 1e5, samples=401)
    assert grid[0] == 2.5 and grid[-1] >= 2.502 > grid[-2]
    assert np.all(np.diff(grid) > 0)
    steps = [G.n_step(n, 2.0, 2000.0, 0.25, 1e5, samples=401) for n in (2.5, 4.0, 7.0)]
    assert steps[0] < steps[1] < steps[2]
    assert G.n_step(4.0, 256.0, 2000.0, 1.0 / 256 ** 2, 1e5, samples=401) > steps[1]


@pytest.mark.parametrize("n", [2.5, 5.0, 7.0])
def test_splice_levels_switch_where_the_spindown_falls_by_four(n):
    f0, t0 = 500.0, 2.0
    lv = G.splice(n, f0, t0, 3)
    k = (1.0 / t0 ** 2) / f0 ** n
    tau = f0 / ((1.0 / t0 ** 2) * (n - 1))
    assert abs(lv[0][1]) < 1e-12 * tau and lv[0][4] == pytest.approx(f0, rel=1e-14)
    for (tf, ta, tb, flo, fhi), nxt in zip(lv, lv[1:] + [None]):
        # spindown of the track at the level's start, by a numerical derivative of Eq. powlaws
        h = max(1e-3, 1e-6 * max(ta, 1.0))
        fd = -(G.power_law_f(ta + h, f0, k, n) - G.power_law_f(max(ta - h, 0.0), f0, k, n)) / (
            ta + h - max(ta - h, 0.0))
        assert fd == pytest.approx(1.0 / tf ** 2, rel=1e-5)
        assert G.power_law_f(tb, f0, k, n) == pytest.approx(flo, rel=1e-12)
        assert flo / fhi == pytest.approx(4.0 ** (-1.0 / n), rel=1e-12)
        if nxt is not None:
            assert nxt[0] == 2 * tf and nxt[1] == pytest.approx(tb, rel=1e-12) and nxt[4] == pytest.approx(flo)
    # tau of Sec. VI.D: the spindown time scale f0 / (fdot0 (n - 1))
    assert lv[1][1] == pytest.approx(tau * (4.0 ** ((n - 1) / n) - 1.0), rel=1e-12)


def test_band_plan_reproduces_the_papers_example_and_covers_the_range():
    # Sec. IV: analysing [200, 300] Hz uses a peakmap of [200, 350] Hz (upper edge x 7/6)
    (a, b, pa, pb), = G.plan_bands(200.0, 300.0, 100.0, 4.0, 1.0 / 6.0, 0.0)
    assert (a, b, pa, pb) == (200.0, 300.0, 200.0, 350.0)
    bands = G.plan_bands(100.0, 2000.0, 64.0, 2.0, 0.2, 8.0)
    assert bands[0][0] == 100.0 and bands[-1][1] == 2000.0
    for (a0, b0, _, _), (a1, b1, _, _) in zip(bands, bands[1:]):
        assert a1 <= b0 and b0 - a1 == pytest.approx(8.0)   # interlaced: every frequency covered
    for a, b, pa, pb in bands:
        assert pa == a and pb >= 1.2 * b - 1e-9 and (pb - 1.2 * b) < 0.5


@pytest.mark.parametrize("n", [2.0, 3.0, 5.0, 7.0])
def test_analysed_columns_are_the_cells_of_the_analysed_band(n):
    # the excluded columns are exactly those whose cell centre inverts (Eq. transform)
    # to a source frequency above the analysed band's top
    f_hi, pm_hi, tfft, pm_lo = 300.0, 350.0, 4.0, 200.0
    df = 1.0 / tfft
    x0_min = pm_hi ** (1 - n)
    dx0 = (n - 1) * df * pm_hi ** (-n)
    n_x0 = int(math.ceil(pm_hi * ((pm_hi / pm_lo) ** (n - 1) - 1) / ((n - 1) * df) - 1e-9))
    lo, hi = G.analysed_columns(n, f_hi, x0_min, dx0, n_x0)
    assert hi == n_x0 and 0 < lo < n_x0
    f_centre = lambda c: (x0_min + (c + 0.5) * dx0) ** (1.0 / (1.0 - n))
    assert f_centre(lo) <= f_hi * (1 + 1e-12) and f_centre(lo - 1) > f_hi * (1 - 1e-12)
    # the same count from the inverse transform: columns between f_hi and pm_hi
    approx = (f_hi ** (1 - n) - x0_min) / dx0
    assert abs(lo - approx) <= 1.0
