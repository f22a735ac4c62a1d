"""Pins of the oracle candidate selection (Sec. IV): closed forms of the
critical ratio, the tie rule, the second-candidate distance, sigma = 0, and
the inverse transform."""
import math

import numpy as np

from oracle import select as OS


def test_single_spike_cr_is_sqrt_n_minus_1():
    # one cell y in a square of N zeros: mu = y/N, sigma = y sqrt(N-1)/N, CR = sqrt(N-1)
    H = np.zeros((6, 10), dtype=np.int32)
    H[2, 7] = 13
    c = OS.select(H, np.arange(6.0), 1.0, 0.1, 3.0, 1, 1, min_dk=0)
    assert len(c) == 1 and (c[0]["row"], c[0]["col"], c[0]["count"]) == (2, 7, 13)
    assert math.isclose(c[0]["cr"], math.sqrt(60 - 1), rel_tol=1e-12)


def test_two_level_square_cr():
    # half the cells a, half b: mu = (a+b)/2, sigma = |a-b|/2, CR of the max = 1
    H = np.zeros((4, 4), dtype=np.int32)
    H[:2] = 9
    H[2:] = 5
    c = OS.select(H, np.ones(4), 1.0, 0.1, 3.0, 1, 1, min_dk=0)
    assert c[0]["cr"] == 1.0 and (c[0]["row"], c[0]["col"]) == (0, 0)  # row-major tie rule


def test_flat_square_gives_no_candidate():
    H = np.full((5, 5), 4, dtype=np.int32)
    assert OS.select(H, np.ones(5), 1.0, 0.1, 3.0, 1, 1) == []


def test_second_candidate_is_min_dk_rows_away():
    rng = np.random.default_rng(0)
    H = rng.integers(0, 5, size=(20, 8)).astype(np.int32)
    H[10, 3] = 50
    H[11, 5] = 49   # too close (1 row)
    H[12, 0] = 48   # 2 rows: too close for min_dk = 3
    H[13, 6] = 47   # 3 rows: the second candidate
    c = OS.select(H, np.arange(20.0), 1.0, 0.1, 3.0, 1, 1, min_dk=3)
    assert [(x["row"], x["col"], x["second"]) for x in c] == [(10, 3, 0), (13, 6, 1)]


def test_squares_partition_the_map_and_columns_range():
    rng = np.random.default_rng(1)
    H = rng.integers(0, 100, size=(17, 23)).astype(np.int32)
    c = OS.select(H, np.arange(17.0), 1.0, 0.1, 3.0, 3, 4, min_dk=0)
    assert len(c) == 12
    for x in c:  # each best lies in its own square and is that square's maximum
        a, b = divmod(x["square"], 4)
        r0, r1 = a * 17 // 3, (a + 1) * 17 // 3
        s0, s1 = b * 23 // 4, (b + 1) * 23 // 4
        assert r0 <= x["row"] < r1 and s0 <= x["col"] < s1
        assert x["count"] == H[r0:r1, s0:s1].max()
    c2 = OS.select(H, np.arange(17.0), 1.0, 0.1, 3.0, 1, 1, min_dk=0, col_lo=5, col_hi=9)
    assert 5 <= c2[0]["col"] < 9 and c2[0]["count"] == H[:, 5:9].max()


def test_candidate_parameters_invert_the_transform(oracle):
    # x0 = f0^(1-n) (Sec. IV, Eq. transform) and k = |fdot0| / f0^n (Sec. II)
    n, f0 = 5.0, 580.0
    x0 = oracle.transform(f0, n)
    dx0 = 1e-17
    col = 37
    x0_min = x0 - (col + 0.5) * dx0
    H = np.zeros((3, 60), dtype=np.int32)
    H[1, col] = 9
    k = np.array([0.0, 2.2e-16, 4.4e-16])
    c = OS.select(H, k, x0_min, dx0, n, 1, 1, min_dk=0)[0]
    assert math.isclose(c["f0"], f0, rel_tol=1e-9)
    assert math.isclose(-c["fdot0"] / c["f0"] ** n, k[1], rel_tol=1e-12)
