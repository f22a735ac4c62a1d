"""Search grids of Sec. VI of the paper, for building plans (host side).

k grid (Sec. VI.B, Eq. dkeqn): the step dk = k((1 + df/f_max)^-n - 1) keeps
the spindown -k f^n of a source at f_max unchanged when its frequency moves by
one bin df = 1/T_FFT, so the grid is geometric with ratio (1 + df/f_max)^-n,
from k_max = fdot_max / f_min^n down to (and just past) k_min = fdot_min /
f_max^n.  Returned ascending, as fh_plan wants, with each point's bin size
k (1 - ratio) for coincidence distances.

n grid (Sec. VI.A): from n_min the step dn is the largest for which the
power-law frequency with n + dn (same f0 and k) stays within one bin of the
one with n over the observation, for the reference source (f0_max,
fdot0_max).  The paper finds dn empirically; here by bisection on a sampled
time axis.

T_FFT splicing (Sec. VI.D): a source starting at f0 with spindown 1/T0^2 is
analysed with T_FFT = T0 until its spindown has fallen by 4, then with 2 T0,
and so on.  Each level is a (T_FFT, time band, frequency band) rectangle.
"""
from __future__ import annotations

import math
from typing import List, NamedTuple, Tuple

import numpy as np


def k_grid(n: float, tfft: float, f_min: float, f_max: float, fdot_min: float,
           fdot_max: float) -> Tuple[np.ndarray, np.ndarray]:
    """(k ascending, bin size of each k)."""
    if not (fdot_min > 0.0 and fdot_max > fdot_min):
        raise ValueError("need 0 < fdot_min < fdot_max")
    if not (0.0 < f_min < f_max and tfft > 0.0):
        raise ValueError("bad band or T_FFT")
    q = (1.0 + (1.0 / tfft) / f_max) ** (-n)
    k_min = fdot_min / f_max ** n
    k_max = fdot_max / f_min ** n
    m = max(0, int(math.ceil(math.log(k_min / k_max) / math.log(q))))
    while k_max * q ** m > k_min:  # guard the rounding of the logarithms
        m += 1
    while m > 0 and k_max * q ** (m - 1) <= k_min:
        m -= 1
    ks = k_max * q ** np.arange(m + 1, dtype=np.float64)
    return ks[::-1].copy(), (ks * (1.0 - q))[::-1].copy()


def power_law(t, f0: float, k: float, n: float):
    """Eq. powlaws."""
    return f0 / (1.0 + k * (n - 1.0) * f0 ** (n - 1.0) * np.asarray(t, dtype=np.float64)) ** (1.0 / (n - 1.0))


def n_step(n: float, tfft: float, f0_max: float, fdot0_max: float, t_obs: float, samples: int = 2001) -> float:
    t = np.linspace(0.0, t_obs, samples)
    k = fdot0_max / f0_max ** n
    f1 = power_law(t, f0_max, k, n)
    df = 1.0 / tfft

    def dev(dn):
        return float(np.max(np.abs(power_law(t, f0_max, k, n + dn) - f1)))

    lo, hi = 0.0, 1e-3
    while dev(hi) <= df:
        lo, hi = hi, hi * 2.0
        if hi > 100.0:
            return hi
    while hi - lo > 1e-6 * hi:
        mid = 0.5 * (lo + hi)
        if dev(mid) <= df:
            lo = mid
        else:
            hi = mid
    return lo


def n_grid(n_min: float, n_max: float, tfft: float, f0_max: float, fdot0_max: float, t_obs: float,
           samples: int = 2001) -> np.ndarray:
    out = [float(n_min)]
    while out[-1] < n_max:
        out.append(out[-1] + n_step(out[-1], tfft, f0_max, fdot0_max, t_obs, samples))
    return np.array(out)


class Level(NamedTuple):
    tfft: float
    t_start: float
    t_end: float
    f_low: float
    f_high: float


def splice(n: float, f0: float, tfft0: float, levels: int) -> List[Level]:
    """Rectangles of Sec. VI.D for the source (f0, fdot0 = 1/T0^2)."""
    # k f^n = 1/T^2 at the start of level l (T = T0 2^l): f_l = f0 4^(-l/n);
    # times from Eq. powlaws with tau = f0 / (fdot0 (n - 1))
    fdot0 = 1.0 / tfft0 ** 2
    tau = f0 / (fdot0 * (n - 1.0))
    out = []
    for lev in range(levels):
        f_hi = f0 * 4.0 ** (-lev / n)
        f_lo = f0 * 4.0 ** (-(lev + 1) / n)
        out.append(Level(tfft0 * 2 ** lev, tau * ((f0 / f_hi) ** (n - 1.0) - 1.0),
                         tau * ((f0 / f_lo) ** (n - 1.0) - 1.0), f_lo, f_hi))
    return out


class Band(NamedTuple):
    f_lo: float   # analysed band [f_lo, f_hi)
    f_hi: float
    pm_lo: float  # peakmap band: the analysed band enlarged at its high edge
    pm_hi: float


def plan_bands(f_start: float, f_stop: float, width: float, tfft: float, enlarge: float = 0.2,
               overlap: float = 0.0) -> List[Band]:
    """Interlaced analysed bands of Sec. IV covering [f_start, f_stop): each is
    `width` Hz (the last one may be shorter), consecutive bands overlap by
    `overlap` Hz, and each peakmap extends the band's top edge by `enlarge`
    times that edge (rounded up to a whole bin), where the transformed noise
    is densest.  Band edges are rounded to whole bins of 1/T_FFT."""
    if not (0 < width and 0 <= overlap < width and f_start < f_stop and enlarge >= 0):
        raise ValueError("bad band plan")
    df = 1.0 / tfft
    out = []
    lo = f_start
    while lo < f_stop - 1e-9:
        hi = min(lo + width, f_stop)
        a = math.floor(lo / df + 1e-9) * df
        b = math.ceil(hi / df - 1e-9) * df
        top = math.ceil(b * (1.0 + enlarge) / df - 1e-9) * df
        out.append(Band(a, b, a, top))
        if hi >= f_stop:
            break
        lo = hi - overlap
    return out


def analysed_columns(n: float, f_hi: float, x0_min: float, dx0: float, n_x0: int) -> Tuple[int, int]:
    """Columns [col_lo, n_x0) of a map whose cell centre x0_min + (c + 0.5) dx0
    lies at or above f_hi^(1-n), i.e. whose source frequency x0^(1/(1-n)) is at
    most f_hi: the candidates of the extra (enlarged) band are left out."""
    X = f_hi ** (1.0 - n)
    c = int(math.ceil((X - x0_min) / dx0 - 0.5))
    c = min(max(c, 0), n_x0)
    while c > 0 and x0_min + (c - 1 + 0.5) * dx0 >= X:
        c -= 1
    while c < n_x0 and x0_min + (c + 0.5) * dx0 < X:
        c += 1
    return c, n_x0
