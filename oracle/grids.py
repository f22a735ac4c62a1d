"""Oracle search grids of Sec. VI (TEST INFRASTRUCTURE ONLY: only tests/, the
smoke check and the benchmark's CPU-baseline leg may import this module).

Plain, slow transcriptions of the paper's grid construction, written from the
equations, one point at a time:

  k grid (Sec. VI.B, Eq. dkeqn): starting at k_max = fdot_max / f_min^n, each
    next point is k + dk with dk = k ((1 + df/f_max)^-n - 1) (negative: the
    grid descends), until k_min = fdot_min / f_max^n is reached or passed.
  n grid (Sec. VI.A, Eqs. dn_powlaws): from n_min, the next braking index is
    n + dn with dn the largest step for which the power-law frequency of
    Eq. powlaws with n + dn stays within one bin df = 1/T_FFT of the one with
    n over the whole observation, for the reference source (f0_max,
    fdot0_max, k = fdot0_max / f0_max^n held fixed), found by bisection.
  T_FFT splicing (Sec. VI.D): the reference source (f0, fdot0 = 1/T0^2) is
    analysed with T_FFT = T0 until its spindown falls by 4, then with 2 T0,
    and so on; level l runs from the time its spindown is 1/T_l^2 to the time
    it is 1/T_{l+1}^2.
"""
import math


def power_law_f(t: float, f0: float, k: float, n: float) -> float:
    """Eq. powlaws: f(t) = f0 / (1 + k (n-1) f0^(n-1) t)^(1/(n-1))."""
    return f0 / (1.0 + k * (n - 1.0) * f0 ** (n - 1.0) * t) ** (1.0 / (n - 1.0))


def k_grid(n: float, tfft: float, f_min: float, f_max: float, fdot_min: float, fdot_max: float):
    """Ascending k grid of Sec. VI.B and the local bin size dk of each point
    (the distance to the next point below it)."""
    if not (fdot_min > 0.0 and fdot_max > fdot_min):
        raise ValueError("need 0 < fdot_min < fdot_max")
    df = 1.0 / tfft
    k_min = fdot_min / f_max ** n
    k_max = fdot_max / f_min ** n
    pts = [k_max]
    while pts[-1] > k_min:
        k = pts[-1]
        dk = k * ((1.0 + df / f_max) ** (-n) - 1.0)
        pts.append(k + dk)
    steps = []
    for i in range(len(pts)):
        k = pts[i]
        steps.append(-k * ((1.0 + df / f_max) ** (-n) - 1.0))
    return list(reversed(pts)), list(reversed(steps))


def max_deviation(n1: float, n2: float, f0: float, k: float, t_obs: float, samples: int = 2001) -> float:
    """max over t in [0, t_obs] of |f(t; n2) - f(t; n1)| at fixed f0 and k."""
    worst = 0.0
    for s in range(samples):
        t = t_obs * s / (samples - 1)
        worst = max(worst, abs(power_law_f(t, f0, k, n2) - power_law_f(t, f0, k, n1)))
    return worst


def n_step(n: float, tfft: float, f0_max: float, fdot0_max: float, t_obs: float, samples: int = 2001) -> float:
    """Largest dn (bisection, relative precision 1e-6) whose frequency
    deviation over t_obs stays within one bin 1/T_FFT."""
    df = 1.0 / tfft
    k = fdot0_max / f0_max ** n
    lo, hi = 0.0, 1e-3
    while max_deviation(n, n + hi, f0_max, k, t_obs, samples) <= df:
        lo, hi = hi, 2.0 * hi
        if hi > 100.0:
            return hi
    while hi - lo > 1e-6 * hi:
        mid = 0.5 * (lo + hi)
        if max_deviation(n, n + mid, f0_max, k, t_obs, samples) <= df:
            lo = mid
        else:
            hi = mid
    return lo


def n_grid(n_min: float, n_max: float, tfft: float, f0_max: float, fdot0_max: float, t_obs: float,
           samples: int = 2001):
    """Braking indices n_min, n_min + dn(n_min), ... up to the first point >= n_max."""
    pts = [n_min]
    while pts[-1] < n_max:
        pts.append(pts[-1] + n_step(pts[-1], tfft, f0_max, fdot0_max, t_obs, samples))
    return pts


def splice(n: float, f0: float, tfft0: float, levels: int):
    """Rectangles (T_FFT, t_start, t_end, f_low, f_high) of Sec. VI.D for the
    reference source f0 with fdot0 = 1/T0^2."""
    k = (1.0 / tfft0 ** 2) / f0 ** n
    out = []
    for lev in range(levels):
        t_l = tfft0 * 2 ** lev
        t_next = 2.0 * t_l
        # spindown k f^n = 1/T^2  ->  f = (1/(T^2 k))^(1/n)
        f_hi = (1.0 / (t_l ** 2 * k)) ** (1.0 / n)
        f_lo = (1.0 / (t_next ** 2 * k)) ** (1.0 / n)
        # invert Eq. powlaws for the times at which f(t) equals those frequencies
        t_a = ((f0 / f_hi) ** (n - 1.0) - 1.0) / (k * (n - 1.0) * f0 ** (n - 1.0))
        t_b = ((f0 / f_lo) ** (n - 1.0) - 1.0) / (k * (n - 1.0) * f0 ** (n - 1.0))
        out.append((t_l, t_a, t_b, f_lo, f_hi))
    return out


def plan_bands(f_start: float, f_stop: float, width: float, tfft: float, enlarge: float, overlap: float):
    """Analysed bands of Sec. IV stepping by width - overlap, each one's peakmap
    band enlarged at the top by enlarge x its upper edge, edges on whole bins."""
    df = 1.0 / tfft
    bands = []
    lo = f_start
    while True:
        hi = min(lo + width, f_stop)
        a = math.floor(lo * tfft + 1e-9) / tfft
        b = math.ceil(hi * tfft - 1e-9) / tfft
        top = math.ceil(b * (1.0 + enlarge) * tfft - 1e-9) / tfft
        bands.append((a, b, a, top))
        if hi >= f_stop:
            return bands
        lo = hi - overlap


def analysed_columns(n: float, f_hi: float, x0_min: float, dx0: float, n_x0: int):
    """Brute force over every column: [first column whose centre's source
    frequency is <= f_hi (compared in x: x0 >= f_hi^(1-n)), n_x0)."""
    X = f_hi ** (1.0 - n)
    for c in range(n_x0):
        if x0_min + (c + 0.5) * dx0 >= X:
            return c, n_x0
    return n_x0, n_x0
