"""Oracle candidate selection (Sec. IV of the paper) -- test infrastructure only.

Squares: rows [floor(a n_k / sq_k), floor((a+1) n_k / sq_k)) x columns
col_lo + [floor(b W / sq_x0), floor((b+1) W / sq_x0)).  In every square the
best cell (largest count; ties: smallest row, then smallest column) is a
candidate, and so is the best cell at least min_dk rows from it.  CR =
(y - mu) / sigma with mu = Sy / N, var = Sy2 / N - mu^2, sigma = sqrt(var)
from exact integer sums (binary64 in that order); sigma = 0 gives none.
Candidate parameters: x0 at the cell centre, k of the row, and the inverse of
the transform x = f^(1-n): f0 = x0^(1/(1-n)), fdot0 = -k f0^n (Sec. II)."""
import math

import numpy as np


def _best(block: np.ndarray, row_ok: np.ndarray):
    """(row, col, y) of the largest count among allowed rows, row-major first."""
    b = np.where(row_ok[:, None], block.astype(np.int64), -1)
    idx = int(np.argmax(b))  # first occurrence in row-major order
    r, c = divmod(idx, block.shape[1])
    return r, c, int(b[r, c])


def select(H: np.ndarray, k, x0_min: float, dx0: float, n: float, sq_k: int, sq_x0: int, min_dk: int = 3,
           cr_thr: float = -math.inf, col_lo: int = 0, col_hi: int = 0):
    n_k, n_x0 = H.shape
    col_hi = col_hi if col_hi > 0 else n_x0
    W = col_hi - col_lo
    out = []
    for a in range(sq_k):
        r0, r1 = (a * n_k) // sq_k, ((a + 1) * n_k) // sq_k
        for b in range(sq_x0):
            s0, s1 = col_lo + (b * W) // sq_x0, col_lo + ((b + 1) * W) // sq_x0
            block = H[r0:r1, s0:s1]
            N = block.size
            if N == 0:
                continue
            Sy = int(block.astype(np.int64).sum())
            Sy2 = int((block.astype(np.int64) ** 2).sum())
            mu = float(Sy) / float(N)
            ex2 = float(Sy2) / float(N)
            var = ex2 - mu * mu
            sigma = math.sqrt(var) if var >= 0 else float("nan")
            if not sigma > 0.0:
                continue
            rows = np.arange(r0, r1)
            picks = []
            br, bc, by = _best(block, np.ones(len(rows), bool))
            picks.append((br, bc, by, 0))
            if min_dk >= 1:
                ok = np.abs(rows - (r0 + br)) >= min_dk
                if ok.any():
                    r2, c2, y2 = _best(block, ok)
                    picks.append((r2, c2, y2, 1))
            for (rr, cc, yy, second) in picks:
                cr = (float(yy) - mu) / sigma
                if not cr >= cr_thr:
                    continue
                row, col = r0 + rr, s0 + cc
                x0 = x0_min + (float(col) + 0.5) * dx0
                f0 = x0 ** (1.0 / (1.0 - n))
                out.append(dict(row=row, col=col, count=yy, square=a * sq_x0 + b, second=second, cr=cr, mu=mu,
                                sigma=sigma, x0=x0, k=float(k[row]), f0=f0, fdot0=-float(k[row]) * f0 ** n))
    return out
