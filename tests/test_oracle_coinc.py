"""Pins of the oracle coincidences (Sec. IV)."""
import math

import numpy as np
import pytest

from oracle import coinc as OC
from oracle import grids as OG


def test_distance_in_bins_and_the_three_bin_window():
    a = [(1.0, 2.0, 0.125, 0.5)]
    # exactly 3 bins in x0 (kept), a hair further (dropped), (2, 3) bins (d = sqrt 13,
    # dropped) and (1.5, 2) bins (d = 2.5, kept); all values exact in binary
    b = [(1.375, 2.0, 0.125, 0.5), (1.375 + 2.0 ** -40, 2.0, 0.125, 0.5), (1.25, 3.5, 0.125, 0.5),
         (1.1875, 3.0, 0.125, 0.5)]
    got = OC.coincide([0, 1], a, [0, 4], b, 3.0)
    assert set(got) == {(0, 0), (0, 3)}
    assert got[(0, 0)] == 3.0 and got[(0, 3)] == 2.5


def test_mean_bin_sizes_make_it_symmetric():
    rng = np.random.default_rng(5)
    a = [tuple(x) for x in np.c_[rng.normal(size=40), rng.normal(size=40), rng.uniform(0.1, 1, 40), rng.uniform(0.1, 1, 40)]]
    b = [tuple(x) for x in np.c_[rng.normal(size=30), rng.normal(size=30), rng.uniform(0.1, 1, 30), rng.uniform(0.1, 1, 30)]]
    ab = OC.coincide([0, 40], a, [0, 30], b, 3.0)
    ba = OC.coincide([0, 30], b, [0, 40], a, 3.0)
    assert {(i, j): d for (i, j), d in ab.items()} == {(j, i): d for (i, j), d in ba.items()}


def test_segments_never_mix():
    a = [(0.0, 0.0, 1.0, 1.0), (0.0, 0.0, 1.0, 1.0)]
    b = [(0.0, 0.0, 1.0, 1.0), (0.0, 0.0, 1.0, 1.0)]
    assert set(OC.coincide([0, 1, 2], a, [0, 1, 2], b, 3.0)) == {(0, 0), (1, 1)}
    assert OC.coincide([0, 2, 2], a, [0, 0, 2], b, 3.0) == {}


@pytest.mark.parametrize("n", [2.5, 3.0, 5.0, 7.0])
def test_line_shift_follows_the_power_law(n):
    # a source seen in an earlier portion, moved by dt along x = x0 + (n-1) k t,
    # lands on x = f(dt)^(1-n) of Eq. powlaws: it coincides with itself later
    f0, k, dt = 700.0, 1e-3 / 700.0 ** n, 3000.0
    f_later = OG.power_law_f(dt, f0, k, n)
    dx0 = 1e-6 * f0 ** (1 - n)
    a = [(f0 ** (1 - n), k, dx0, k * 1e-3)]
    b = [(f_later ** (1 - n), k, dx0, k * 1e-3)]
    got = OC.coincide([0, 1], a, [0, 1], b, 3.0, nm1=[n - 1], dt=[dt])
    assert got[(0, 0)] < 1e-3
    assert OC.coincide([0, 1], a, [0, 1], b, 3.0) == {}  # without the shift they are far apart
