"""Oracle of the tile CNN -- test infrastructure only.

Plain numpy, float64.  With `bf16=True` it rounds (to nearest even, through
float32) at the same points as the GPU network: input tiles, conv weights,
every ReLU output and every activation gradient; with `bf16=False` it is the
exact float64 network, whose gradients the tests check against central
finite differences.

Network: 4 x [3x3 conv, zero padding, bias, ReLU] 1 -> 16 -> 32 -> 64 -> 64,
global average pool, linear 64 -> 1, logistic; loss = mean binary
cross-entropy; the optimiser is Adam (adam_step).  Parameter vector order: w1 [16][9], b1, w2 [32][9][16], b2,
w3 [64][9][32], b3, w4 [64][9][64], b4, w5 [64], b5 (conv weight index
[co][dy*3+dx][ci])."""
import numpy as np

CH = [1, 16, 32, 64, 64]
HW = 64


def bf16(a):
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return (u & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for l in range(4):
        ci, co = CH[l], CH[l + 1]
        n = co * 9 * ci
        out[f"w{l + 1}"] = theta[o:o + n].reshape(co, 9, ci)
        o += n
        out[f"b{l + 1}"] = theta[o:o + co]
        o += co
    out["w5"] = theta[o:o + 64]
    out["b5"] = theta[o + 64]
    assert o + 65 == theta.size == 60289
    return out


def _conv(x, w, b):
    """x (B, 64, 64, Cin), w (Cout, 9, Cin): zero-padded 3x3 correlation + bias."""
    B = x.shape[0]
    xp = np.zeros((B, HW + 2, HW + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((B, HW, HW, w.shape[0])) + b
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        out += xp[:, dy:dy + HW, dx:dx + HW, :] @ w[:, tap, :].T
    return out


def _conv_data_grad(d, w):
    """Gradient of _conv's output d (B, 64, 64, Cout) w.r.t. its input."""
    B = d.shape[0]
    dp = np.zeros((B, HW + 2, HW + 2, d.shape[3]))
    dp[:, 1:-1, 1:-1] = d
    out = np.zeros((B, HW, HW, w.shape[2]))
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        out += dp[:, 2 - dy:2 - dy + HW, 2 - dx:2 - dx + HW, :] @ w[:, tap, :]
    return out


def _conv_weight_grad(x, d):
    """dW (Cout, 9, Cin) and db of _conv for input x and output gradient d."""
    B = x.shape[0]
    xp = np.zeros((B, HW + 2, HW + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1] = x
    dw = np.zeros((d.shape[3], 9, x.shape[3]))
    dflat = d.reshape(-1, d.shape[3])
    for tap in range(9):
        dy, dx = divmod(tap, 3)
        dw[:, tap, :] = dflat.T @ xp[:, dy:dy + HW, dx:dx + HW, :].reshape(-1, x.shape[3])
    return dw, dflat.sum(0)


def forward(theta, tiles, bf=True):
    """tiles (B, 64, 64) -> (logits (B,), cache)."""
    P = unpack(theta)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    a = [r(np.asarray(tiles, dtype=np.float64))[..., None]]
    for l in range(1, 5):
        z = _conv(a[-1], r(P[f"w{l}"]), P[f"b{l}"])
        a.append(r(np.maximum(z, 0.0)))
    feat = a[4].mean(axis=(1, 2))
    logit = feat @ P["w5"] + P["b5"]
    return logit, dict(P=P, a=a, feat=feat, bf=bf)


def loss_and_grad(theta, tiles, labels, bf=True):
    logit, c = forward(theta, tiles, bf)
    P, a, feat = c["P"], c["a"], c["feat"]
    r = bf16 if bf else (lambda v: v)
    y = np.asarray(labels, dtype=np.float64)
    B = len(y)
    loss = np.mean(np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit))))
    dz = (1.0 / (1.0 + np.exp(-logit)) - y) / B
    g = {"w5": dz @ feat, "b5": dz.sum()}
    d = r((dz[:, None, None, None] * P["w5"][None, None, None, :]) * (1.0 / (HW * HW)) * (a[4] > 0))
    for l in range(4, 0, -1):
        g[f"w{l}"], g[f"b{l}"] = _conv_weight_grad(a[l - 1], d)
        if l > 1:
            d = r(_conv_data_grad(d, r(P[f"w{l}"])) * (a[l - 1] > 0))
    flat = np.concatenate([np.concatenate([g[f"w{l}"].ravel(), g[f"b{l}"].ravel()]) for l in range(1, 5)] +
                          [g["w5"].ravel(), np.atleast_1d(g["b5"])])
    return loss, flat, logit


def init_params(rng, scale=1.0):
    """He-normal conv weights, zero biases, small head."""
    th = []
    for l in range(4):
        ci, co = CH[l], CH[l + 1]
        th.append(rng.normal(0, scale * np.sqrt(2.0 / (9 * ci)), co * 9 * ci))
        th.append(np.zeros(co))
    th.append(rng.normal(0, 0.1, 64))
    th.append(np.zeros(1))
    return np.concatenate(th)


def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015, the algorithm of their
    Sec. 2) in float64: moving averages of the gradient and of its square,
    each divided by its bias correction 1 - beta^t, then a step of lr times
    the corrected mean over (square root of the corrected second moment plus
    eps).  t counts steps from 1.  Returns new (theta, m, v); inputs are not
    modified."""
    g = np.asarray(grad, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * (g * g)
    m_hat = m / (1.0 - b1 ** t)
    v_hat = v / (1.0 - b2 ** t)
    theta = np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v
