"""ctypes wrapper of the C oracle (fh_oracle.c) -- test infrastructure only.

The C file states the method and the canonical FP64 form; this wrapper only
marshals numpy arrays.  Built by oracle/build.py (gcc, -ffp-contract=off,
OpenMP over k rows)."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_fh.so")


class OrcDesc(C.Structure):
    _fields_ = [("n", C.c_double), ("tfft", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double),
                ("n_fft", C.c_int32), ("t", C.POINTER(C.c_double)), ("n_k", C.c_int32),
                ("k", C.POINTER(C.c_double)), ("x0_min", C.c_double), ("dx0", C.c_double),
                ("n_x0", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build
            build.build()
        L = C.CDLL(LIB_PATH)
        L.orc_n_freq.restype = C.c_int
        L.orc_n_freq.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_transform.restype = C.c_double
        L.orc_transform.argtypes = [C.c_double, C.c_double]
        L.orc_x0_grid.restype = None
        L.orc_x0_grid.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_n_x0.restype = C.c_int
        L.orc_n_x0.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
        dp = C.POINTER(C.c_double)
        L.orc_tables.restype = None
        L.orc_tables.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double, C.c_int, dp,
                                 C.c_int, dp, dp, dp, dp]
        ip = C.POINTER(C.c_int32)
        L.orc_hough_rows.restype = C.c_int
        L.orc_hough_rows.argtypes = [C.POINTER(OrcDesc), ip, ip, ip, C.c_int32, ip, C.POINTER(C.c_int64)]
        L.orc_hough_rows_pairs.restype = C.c_int
        L.orc_hough_rows_pairs.argtypes = [C.POINTER(OrcDesc), ip, ip, ip, C.c_int32, ip, C.POINTER(C.c_int64),
                                           C.POINTER(C.c_int64)]
        L.orc_rows_checked.restype = C.c_int
        L.orc_rows_checked.argtypes = [C.POINTER(OrcDesc), ip, ip, ip, C.c_int32, ip, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64)]
        L.orc_pair_interval.restype = C.c_int
        L.orc_pair_interval.argtypes = [C.POINTER(OrcDesc), C.c_int32, C.c_int32, C.c_int32, ip, ip]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        _lib = L
    return _lib


def threads() -> int:
    """Threads the oracle's row loop uses."""
    return int(lib().orc_threads())


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_double)()
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: Optional[np.ndarray]):
    if a is None:
        return C.POINTER(C.c_int32)()
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Desc:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, n, tfft, f_min, f_max, n_fft, k, t=None, x0_min=0.0, dx0=0.0, n_x0=0):
        self.k = np.ascontiguousarray(k, dtype=np.float64)
        self.t = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
        self.c = OrcDesc(float(n), float(tfft), float(f_min), float(f_max), int(n_fft), _dptr(self.t),
                         int(self.k.shape[0]), _dptr(self.k), float(x0_min), float(dx0), int(n_x0))

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec.n, spec.tfft, spec.f_min, spec.f_max, spec.n_fft, spec.k, **kw)

    @property
    def n_k(self):
        return int(self.c.n_k)


def n_freq(tfft, f_min, f_max) -> int:
    return lib().orc_n_freq(tfft, f_min, f_max)


def transform(f: float, n: float) -> float:
    return lib().orc_transform(f, n)


def x0_grid(n, tfft, f_max):
    a, b = C.c_double(), C.c_double()
    lib().orc_x0_grid(n, tfft, f_max, C.byref(a), C.byref(b))
    return a.value, b.value


def n_x0(n, tfft, f_min, f_max) -> int:
    return lib().orc_n_x0(n, tfft, f_min, f_max)


def grid(d: Desc):
    """(n_f, x0_min, dx0, n_x0) exactly as the oracle resolves them."""
    c = d.c
    nf = n_freq(c.tfft, c.f_min, c.f_max)
    if c.dx0 != 0.0:
        x0m, dx = c.x0_min, c.dx0
    else:
        x0m, dx = x0_grid(c.n, c.tfft, c.f_max)
    nx = c.n_x0 if c.n_x0 > 0 else n_x0(c.n, c.tfft, c.f_min, c.f_max)
    return nf, x0m, dx, nx


def tables(d: Desc):
    nf, x0m, dx, nx = grid(d)
    c = d.c
    A = np.empty(nf + 1)
    Cr = np.empty(max(1, c.n_k))
    T = np.empty(max(1, c.n_fft))
    lib().orc_tables(c.n, c.tfft, c.f_min, nf, x0m, dx, c.n_k, _dptr(d.k), c.n_fft, _dptr(d.t), _dptr(A),
                     _dptr(Cr), _dptr(T))
    return A, Cr[:c.n_k], T[:c.n_fft]


def hough(d: Desc, row_ptr: np.ndarray, bin_: np.ndarray, rows: Optional[Sequence[int]] = None,
          return_bad: bool = False, return_pairs: bool = False):
    """Direct Hough map, int32 [n_rows][n_x0] (all rows if rows is None);
    with return_bad / return_pairs also the count of skipped bad peaks and of
    (row, peak) pairs whose clipped interval holds a column."""
    nf, x0m, dx, nx = grid(d)
    if nf < 0 or nx <= 0:
        raise ValueError("invalid map description")
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    bn = np.ascontiguousarray(bin_, dtype=np.int32)
    assert rp.shape[0] == d.c.n_fft + 1
    rl = None if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    nr = d.n_k if rl is None else rl.shape[0]
    out = np.empty((nr, nx), dtype=np.int32)
    bad = C.c_int64(0)
    pairs = C.c_int64(0)
    st = lib().orc_hough_rows_pairs(C.byref(d.c), _iptr(rp), _iptr(bn), _iptr(rl), 0 if rl is None else nr,
                                    _iptr(out), C.byref(bad), C.byref(pairs))
    if st != 0:
        raise ValueError("oracle rejected the description")
    extra = ((bad.value,) if return_bad else ()) + ((pairs.value,) if return_pairs else ())
    return (out,) + extra if extra else out


def rows_checked(d: Desc, row_ptr: np.ndarray, bin_: np.ndarray, rows: Sequence[int], with_map: bool = True):
    """(map rows int32 [len(rows)][n_x0] or None, row totals int64, in-grid pairs
    int64) of the listed rows, from orc_rows_checked (direct counting with the
    early exits the ordering of the peaks allows)."""
    nf, x0m, dx, nx = grid(d)
    if nf < 0 or nx <= 0:
        raise ValueError("invalid map description")
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    bn = np.ascontiguousarray(bin_, dtype=np.int32)
    assert rp.shape[0] == d.c.n_fft + 1
    rl = np.ascontiguousarray(rows, dtype=np.int32)
    assert rl.size == 0 or (rl.min() >= 0 and rl.max() < d.n_k)
    out = np.empty((rl.shape[0], nx), dtype=np.int32) if with_map else None
    tot = np.empty(rl.shape[0], dtype=np.int64)
    prs = np.empty(rl.shape[0], dtype=np.int64)
    st = lib().orc_rows_checked(C.byref(d.c), _iptr(rp), _iptr(bn), _iptr(rl), rl.shape[0], _iptr(out),
                                tot.ctypes.data_as(C.POINTER(C.c_int64)), prs.ctypes.data_as(C.POINTER(C.c_int64)))
    if st != 0:
        raise ValueError("oracle rejected the description")
    return out, tot, prs


def pair_interval(d: Desc, r: int, i: int, j: int):
    lo, hi = C.c_int32(), C.c_int32()
    w = lib().orc_pair_interval(C.byref(d.c), r, i, j, C.byref(lo), C.byref(hi))
    return lo.value, hi.value, w
