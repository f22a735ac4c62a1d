"""Oracle coincidences (Sec. IV) -- TEST INFRASTRUCTURE ONLY.

Two candidate lists, grouped in segments; every pair (a, b) of one segment is
checked by brute force: a is first moved along its line x = x0 + (n-1) k t by
the segment's dt (Eq. transform: x0' = x0 + ((n-1) k) dt), then
  d = sqrt(u^2 + v^2), u = (x0_b - x0_a') / ((dx0_a + dx0_b) / 2),
                       v = (k_b - k_a) / ((dk_a + dk_b) / 2)
(binary64, this order), and the pair is kept when d <= max_d."""
import math


def coincide(a_off, a, b_off, b, max_d, nm1=None, dt=None):
    """a, b: sequences of (x0, k, dx0, dk).  Returns {(ia, ib): d}."""
    out = {}
    n_seg = len(a_off) - 1
    for s in range(n_seg):
        for ia in range(a_off[s], a_off[s + 1]):
            x0a, ka, dxa, dka = (float(v) for v in a[ia])
            if nm1 is not None and dt is not None:
                x0a = x0a + (float(nm1[s]) * ka) * float(dt[s])
            for ib in range(b_off[s], b_off[s + 1]):
                x0b, kb, dxb, dkb = (float(v) for v in b[ib])
                u = (x0b - x0a) / ((dxa + dxb) * 0.5)
                v = (kb - ka) / ((dka + dkb) * 0.5)
                d = math.sqrt(u * u + v * v)
                if d <= max_d:
                    out[(ia, ib)] = d
    return out
