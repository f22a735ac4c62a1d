"""Oracle follow-up on peakmaps (Sec. V) -- TEST INFRASTRUCTURE ONLY.

roi_grid: the coarse cell's +-half bins re-gridded `over` times finer.
project: every peak (i, j) moved by the candidate's drift,
  j -> j - (b_i - b_0),  b_i = floor((f(T_i) - f_min) tfft),  b_0 = floor((f0 - f_min) tfft),
  f(T) = f0 / (1 + ((k (n-1)) f0^(n-1)) T)^(1/(n-1))   (Eq. powlaws),
then counted per moved bin within b_0 +- w; the bin b_0 gets CR = (y - mu) / sigma
against the bins outside b_0 +- guard (population statistics from exact sums,
binary64, this order; sigma = 0 gives NaN)."""
import math


def roi_grid(x0_c, k_c, dx0, dk, over=10, half=3):
    m = 2 * half * over
    ks = []
    for i in range(m):
        k = k_c + (dk / over) * (i - half * over)
        if k >= 0.0:
            ks.append(k)
    return x0_c - half * dx0, dx0 / over, m, ks


def project(row_ptr, bins, T, n, tfft, f_min, n_f, f0, k, w, guard):
    nm1 = n - 1.0
    a = (k * nm1) * f0 ** nm1
    b0 = math.floor((f0 - f_min) * tfft)
    hist = [0] * (2 * w + 1)
    for i in range(len(row_ptr) - 1):
        f = f0 / (1.0 + a * T[i]) ** (1.0 / nm1)
        shift = math.floor((f - f_min) * tfft) - b0
        for p in range(row_ptr[i], row_ptr[i + 1]):
            j = int(bins[p])
            if not 0 <= j < n_f:
                continue
            d = j - shift - b0
            if -w <= d <= w:
                hist[d + w] += 1
    S = S2 = N = 0
    for x, y in enumerate(hist):
        if w - guard <= x <= w + guard:
            continue
        S += y
        S2 += y * y
        N += 1
    mu = S / N
    var = S2 / N - mu * mu
    sigma = math.sqrt(var) if var >= 0 else float("nan")
    y0 = hist[w]
    cr = (y0 - mu) / sigma if sigma > 0 else float("nan")
    return hist, {"y": y0, "mu": mu, "sigma": sigma, "cr": cr}
