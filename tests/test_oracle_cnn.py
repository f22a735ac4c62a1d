"""Pins of the CNN oracle: exact float64 gradients against central finite
differences, the BF16 rounding rule, and the layer algebra on closed forms."""
import numpy as np

from oracle import cnn as N


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38, 1e-40])
    got = N.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1; 1 + 3*2^-8 -> 1 + 2^-6
    assert list(got[:4]) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6]
    assert got[4] == -2.5
    assert np.all(np.abs(N.bf16(np.linspace(-3, 3, 1001)) - np.linspace(-3, 3, 1001)) <=
                  np.abs(np.linspace(-3, 3, 1001)) * 2 ** -8 + 1e-300)


def test_conv_is_a_correlation_with_zero_padding():
    # a single nonzero input pixel reproduces the flipped kernel around it
    x = np.zeros((1, 64, 64, 1))
    x[0, 10, 20, 0] = 1.0
    w = np.arange(9, dtype=np.float64).reshape(1, 9, 1)
    y = N._conv(x, w, np.zeros(1))
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        assert y[0, 10 - dy + 1, 20 - dx + 1, 0] == tap
    assert y.sum() == w.sum()
    # corner pixel: the taps that leave the tile see zeros
    x = np.zeros((1, 64, 64, 1))
    x[0, 0, 0, 0] = 1.0
    assert N._conv(x, w, np.zeros(1)).sum() == w[0, [0, 1, 3, 4], 0].sum()


def test_data_and_weight_gradients_are_adjoint():
    # <conv(x, w), d> = <x, conv_data_grad(d, w)> = <w, conv_weight_grad(x, d)>
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 64, 64, 3))
    w = rng.normal(size=(4, 9, 3))
    d = rng.normal(size=(2, 64, 64, 4))
    lhs = np.sum(N._conv(x, w, np.zeros(4)) * d)
    assert np.isclose(lhs, np.sum(x * N._conv_data_grad(d, w)), rtol=1e-10)
    dw, db = N._conv_weight_grad(x, d)
    assert np.isclose(lhs, np.sum(w * dw), rtol=1e-10)
    assert np.allclose(db, d.sum(axis=(0, 1, 2)))


def test_exact_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    th = N.init_params(rng)
    tiles = rng.normal(size=(2, 64, 64))
    labels = np.array([1.0, 0.0])
    loss, g, _ = N.loss_and_grad(th, tiles, labels, bf=False)
    idx = np.concatenate([rng.choice(np.arange(0, 160), 6, replace=False),       # conv1
                          rng.choice(np.arange(160, 4800), 6, replace=False),    # conv2
                          rng.choice(np.arange(4800, 23296), 6, replace=False),  # conv3
                          rng.choice(np.arange(23296, 60224), 6, replace=False),  # conv4
                          [60224, 60240, 60288]])                                # head
    for i in idx:
        errs = []
        for h in (1e-6, 3e-7):  # small steps: a ReLU kink inside the step spoils larger ones
            tp, tm = th.copy(), th.copy()
            tp[i] += h
            tm[i] -= h
            fd = (N.loss_and_grad(tp, tiles, labels, bf=False)[0] -
                  N.loss_and_grad(tm, tiles, labels, bf=False)[0]) / (2 * h)
            errs.append(abs(fd - g[i]) / (abs(g[i]) + 1e-4))  # + roundoff of the differences
        assert min(errs) <= 1e-5, (i, errs, g[i])


def test_parameter_count():
    assert N.init_params(np.random.default_rng(0)).size == 60289
