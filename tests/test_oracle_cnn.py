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


# --- the optimiser (Adam, Kingma and Ba 2015) -------------------------------

def _run_adam(grads, lr, p0=None, **kw):
    p = np.zeros(grads[0].shape) if p0 is None else np.array(p0, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    out = []
    for t, g in enumerate(grads, start=1):
        p, m, v = N.adam_step(p, g, m, v, t, lr, **kw)
        out.append(p.copy())
    return out


def test_adam_first_step_moves_by_lr_times_sign():
    # from zero moments the corrected mean is g and the corrected second moment
    # g^2, so the first step is lr * g / (|g| + eps): about lr in the direction -g
    g = np.array([3.0, -0.5, 1e-3, -2e-6, 0.0])
    (p1,) = _run_adam([g], lr=0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=0)
    assert np.allclose(p1[:3], [-0.01, 0.01, -0.01], rtol=1e-4)
    assert p1[4] == 0.0


def test_adam_constant_gradient_moves_linearly():
    # a constant gradient keeps both corrected moments at g and g^2 for every t
    g = np.array([0.7, -4.0, 2.5e-3])
    ps = _run_adam([g] * 12, lr=2e-3, p0=[1.0, 2.0, 3.0])
    for t, p in enumerate(ps, start=1):
        assert np.allclose(p, np.array([1.0, 2.0, 3.0]) - t * 2e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_zero_gradient_and_symmetries():
    rng = np.random.default_rng(11)
    grads = [rng.normal(size=40) * 10.0 ** rng.uniform(-6, 1, 40) for _ in range(7)]
    base = _run_adam(grads, lr=1e-3)
    # negating every gradient negates the path
    neg = _run_adam([-g for g in grads], lr=1e-3)
    assert all(np.allclose(a, -b, rtol=1e-12, atol=0) for a, b in zip(base, neg))
    # with eps = 0 the update does not depend on the gradients' scale
    s0 = _run_adam(grads, lr=1e-3, eps=0.0)
    s1 = _run_adam([37.0 * g for g in grads], lr=1e-3, eps=0.0)
    assert all(np.allclose(a, b, rtol=1e-12, atol=1e-18) for a, b in zip(s0, s1))
    # but with eps > 0 tiny gradients move less than large ones (eps is outside the root)
    tiny = _run_adam([np.full(3, 1e-9)], lr=1.0)[0]
    assert np.allclose(tiny, -1e-9 / (1e-9 + 1e-8), rtol=1e-12)
    # a zero gradient never moves a parameter, before or after other steps
    zero = _run_adam([np.zeros(5)] * 4, lr=0.1, p0=np.arange(5.0))
    assert all(np.array_equal(p, np.arange(5.0)) for p in zero)


def test_adam_impulse_response():
    # a single unit gradient at step 1, zeros after: the moments decay
    # geometrically, m_t = b^(t-1) (1 - b) for each average, so the corrected
    # ratio at step t is b1^(t-1)(1-b1)/(1-b1^t) over the root of
    # b2^(t-1)(1-b2)/(1-b2^t) (this separates the roles of b1 and b2)
    b1, b2, lr = 0.9, 0.999, 1e-2
    ps = _run_adam([np.ones(1)] + [np.zeros(1)] * 9, lr=lr)
    prev = 0.0
    for t, p in enumerate(ps, start=1):
        mh = b1 ** (t - 1) * (1 - b1) / (1 - b1 ** t)
        vh = b2 ** (t - 1) * (1 - b2) / (1 - b2 ** t)
        assert np.isclose(prev - p[0], lr * mh / (np.sqrt(vh) + 1e-8), rtol=1e-12)
        prev = p[0]
