"""Thin ctypes binding of libfh.so (the C ABI in include/fh.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's kernels.  The
library must have been built (paper_1810_09784_amd/build.py); there is no
fallback of any kind."""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfh.so")

FH_OK, FH_EINVAL, FH_ENOMEM, FH_EDEVICE, FH_ERANGE = 0, -1, -2, -3, -4


class FHError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_str(status)} ({status})")
        self.status = status


class MapDesc(C.Structure):
    _fields_ = [("n", C.c_double), ("tfft", C.c_double), ("f_min", C.c_double), ("f_max", C.c_double),
                ("n_fft", C.c_int32), ("t", C.POINTER(C.c_double)), ("n_k", C.c_int32),
                ("k", C.POINTER(C.c_double)), ("x0_min", C.c_double), ("dx0", C.c_double), ("n_x0", C.c_int32)]


class Peaks(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("bin", C.c_void_p), ("n_peaks", C.c_int64)]


class TileCfg(C.Structure):
    _fields_ = [("rows", C.c_int32), ("cols", C.c_int32), ("threads", C.c_int32), ("mode", C.c_int32),
                ("tsplit", C.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class SelectOpts(C.Structure):
    _fields_ = [("sq_k", C.c_int32), ("sq_x0", C.c_int32), ("min_dk", C.c_int32), ("col_lo", C.c_int32),
                ("col_hi", C.c_int32), ("cr_thr", C.c_double)]


class Candidate(C.Structure):
    _fields_ = [("row", C.c_int32), ("col", C.c_int32), ("count", C.c_int32), ("square", C.c_int32),
                ("second", C.c_int32), ("pad", C.c_int32), ("cr", C.c_double), ("mu", C.c_double),
                ("sigma", C.c_double), ("x0", C.c_double), ("k", C.c_double), ("f0", C.c_double),
                ("fdot0", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class Projection(C.Structure):
    _fields_ = [("y", C.c_int32), ("host_drift", C.c_int32), ("mu", C.c_double), ("sigma", C.c_double),
                ("cr", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("n_f", C.c_int32), ("n_x0", C.c_int32), ("n_k", C.c_int32), ("n_fft", C.c_int32),
                ("x0_min", C.c_double), ("dx0", C.c_double), ("tile", TileCfg), ("n_tiles", C.c_int64),
                ("workspace_bytes", C.c_int64)]


_lib = None

# name -> (restype, argtypes); every symbol include/fh.h declares
SIGNATURES = {
    "fh_plan": (C.c_int, [C.POINTER(MapDesc), C.POINTER(TileCfg), C.POINTER(C.c_void_p)]),
    "fh_plan_get_info": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "fh_plan_tables": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "fh_plan_destroy": (None, [C.c_void_p]),
    "fh_hough": (C.c_int, [C.c_void_p, C.POINTER(Peaks), C.c_void_p, C.c_void_p]),
    "fh_hough_select": (C.c_int, [C.c_void_p, C.POINTER(Peaks), C.c_void_p, C.POINTER(SelectOpts), C.c_void_p]),
    "fh_select_results": (C.c_int, [C.c_void_p, C.POINTER(Candidate), C.c_int32, C.POINTER(C.c_int32)]),
    "fh_device_errors": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]),
    "fh_plan_set_events": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fh_batch_create": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(Peaks), C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_void_p)]),
    "fh_batch_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fh_batch_launch_plain": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fh_batch_destroy": (None, [C.c_void_p]),
    "fh_hough_batched": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(Peaks), C.POINTER(C.c_void_p),
                                   C.c_void_p]),
    "fh_batch_select": (C.c_int, [C.c_void_p, C.POINTER(SelectOpts), C.POINTER(Candidate), C.c_int32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_void_p]),
    "fh_batch_propose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p,
                                   C.c_void_p]),
    "fh_peaks_validate": (C.c_int, [C.c_void_p]),
    "fh_select_tiles": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SelectOpts), C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_int32, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "fh_batch_select_tiles": (C.c_int, [C.c_void_p, C.POINTER(SelectOpts), C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_int32, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p]),
    "fh_select": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SelectOpts), C.c_void_p, C.c_int32,
                            C.POINTER(C.c_int32), C.c_void_p]),
    "fh_select_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(SelectOpts), C.c_void_p, C.c_int32,
                            C.POINTER(C.c_int32), C.c_void_p]),
    "fh_cnn_create": (C.c_int, [C.c_int32, C.POINTER(C.c_void_p)]),
    "fh_cnn_destroy": (None, [C.c_void_p]),
    "fh_cnn_num_params": (C.c_int64, []),
    "fh_cnn_set_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "fh_cnn_get_params": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "fh_cnn_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "fh_cnn_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "fh_cnn_step": (C.c_int, [C.c_void_p, C.c_float, C.c_void_p]),
    "fh_cnn_set_grads": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "fh_cnn_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "fh_cnn_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64]),
    "fh_cnn_scores": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "fh_cnn_activations": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "fh_tiles": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "fh_propose": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "fh_coincide": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                              C.c_void_p]),
    "fh_project": (C.c_int, [C.c_void_p, C.POINTER(Peaks), C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                             C.c_void_p, C.c_void_p, C.c_void_p]),
    "fh_status_str": (C.c_char_p, [C.c_int]),
    "fh_version": (C.c_char_p, []),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1810_09784_amd/build.py "
                               "(or __graft_entry__.build())")
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()  # one HIP runtime (torch's) initialised before the library's first call
            torch.zeros(1, device="cuda")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_str(s: int) -> str:
    return lib().fh_status_str(int(s)).decode()


def _check(st: int, what: str):
    if st != FH_OK:
        raise FHError(st, what)


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(int(stream.cuda_stream))


def _ptr(t) -> int:
    return int(t.data_ptr())


class Plan:
    """fh_plan: a validated map description with its device tables."""

    def __init__(self, n: float, tfft: float, f_min: float, f_max: float, n_fft: int, k: Sequence[float],
                 t: Optional[Sequence[float]] = None, x0_min: float = 0.0, dx0: float = 0.0, n_x0: int = 0,
                 tile: Optional[dict] = None):
        self._k = np.ascontiguousarray(k, dtype=np.float64)
        self._t = None if t is None else np.ascontiguousarray(t, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self.desc = MapDesc(float(n), float(tfft), float(f_min), float(f_max), int(n_fft),
                            dp() if self._t is None else self._t.ctypes.data_as(dp), int(self._k.shape[0]),
                            self._k.ctypes.data_as(dp), float(x0_min), float(dx0), int(n_x0))
        cfg = None
        if tile:
            cfg = TileCfg(int(tile.get("rows", 0)), int(tile.get("cols", 0)), int(tile.get("threads", 0)),
                          int(tile.get("mode", 0)), int(tile.get("tsplit", 1)))
        h = C.c_void_p()
        _check(lib().fh_plan(C.byref(self.desc), C.byref(cfg) if cfg else None, C.byref(h)), "fh_plan")
        self.handle = h
        info = PlanInfo()
        _check(lib().fh_plan_get_info(h, C.byref(info)), "fh_plan_get_info")
        self.info = info

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec.n, spec.tfft, spec.f_min, spec.f_max, spec.n_fft, spec.k, **kw)

    @property
    def n_k(self):
        return int(self.info.n_k)

    @property
    def n_x0(self):
        return int(self.info.n_x0)

    @property
    def n_f(self):
        return int(self.info.n_f)

    @property
    def tile(self):
        return self.info.tile.as_dict()

    def tables(self):
        A = np.empty(self.n_f + 1)
        Cr = np.empty(self.n_k)
        T = np.empty(int(self.info.n_fft))
        _check(lib().fh_plan_tables(self.handle, A.ctypes.data, Cr.ctypes.data, T.ctypes.data), "fh_plan_tables")
        return A, Cr, T

    def destroy(self):
        if self.handle:
            lib().fh_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fh_plan(*args, **kw) -> Plan:
    return Plan(*args, **kw)


def peaks_struct(row_ptr, bin_) -> Peaks:
    """row_ptr / bin: int32 CUDA tensors (CSR by FFT)."""
    import torch
    assert row_ptr.is_cuda and bin_.is_cuda and row_ptr.dtype == torch.int32 and bin_.dtype == torch.int32
    assert row_ptr.is_contiguous() and bin_.is_contiguous()
    return Peaks(_ptr(row_ptr), _ptr(bin_) if bin_.numel() else 0, int(bin_.numel()))


def fh_hough(plan: Plan, row_ptr, bin_, out=None, stream=None):
    """Hough map of one peakmap; returns (or fills) an int32 [n_k, n_x0] CUDA tensor."""
    import torch
    if out is None:
        out = torch.empty((plan.n_k, plan.n_x0), dtype=torch.int32, device=row_ptr.device)
    assert out.dtype == torch.int32 and out.is_contiguous() and tuple(out.shape) == (plan.n_k, plan.n_x0)
    if row_ptr.numel() != int(plan.info.n_fft) + 1:
        raise ValueError("row_ptr must have n_fft + 1 entries")
    pk = peaks_struct(row_ptr, bin_)
    _check(lib().fh_hough(plan.handle, C.byref(pk), C.c_void_p(_ptr(out)), _stream(stream)), "fh_hough")
    return out


def fh_plan_set_events(plan: Plan, start=None, stop=None):
    """start/stop: torch.cuda.Event(enable_timing=True) or None (clears)."""
    a = C.c_void_p(int(start.cuda_event)) if start is not None else None
    b = C.c_void_p(int(stop.cuda_event)) if stop is not None else None
    _check(lib().fh_plan_set_events(plan.handle, a, b), "fh_plan_set_events")


def fh_device_errors(plan: Plan, stream=None) -> int:
    v = C.c_uint64()
    _check(lib().fh_device_errors(plan.handle, _stream(stream), C.byref(v)), "fh_device_errors")
    return int(v.value)


def fh_select(plan: Plan, hmap, sq_k: int, sq_x0: int, min_dk: int = 3, cr_thr: float = -1e300,
              col_lo: int = 0, col_hi: int = 0, cap: int = None, stream=None, as_dicts: bool = True):
    """Candidates of a Hough map in square order: (list of dicts, total) or, with
    as_dicts=False, (numpy structured array of the returned records, total).
    cap defaults to 2 sq_k sq_x0, the most the selection can return."""
    assert hmap.is_cuda and tuple(hmap.shape) == (plan.n_k, plan.n_x0) and hmap.is_contiguous()
    if cap is None:
        cap = 2 * int(sq_k) * int(sq_x0)
    opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
    buf = (Candidate * max(1, cap))()
    n = C.c_int32()
    _check(lib().fh_select(plan.handle, C.c_void_p(_ptr(hmap)), C.byref(opts), buf, int(cap), C.byref(n),
                           _stream(stream)), "fh_select")
    m = min(n.value, cap)
    if not as_dicts:
        import numpy as np
        return np.ctypeslib.as_array(buf)[:m].copy(), int(n.value)
    return [buf[i].as_dict() for i in range(m)], int(n.value)


def fh_select_tiles(plan: Plan, hmap, tiles: Sequence[int], sq_k: int, sq_x0: int, min_dk: int = 3,
                    cr_thr: float = -1e300, col_lo: int = 0, col_hi: int = 0, cap: int = None, stream=None,
                    as_dicts: bool = True):
    """The selection inside the listed 64 x 64 tiles only, each with its own
    squares and statistics: (candidates, per-tile counts, total)."""
    import numpy as np
    assert hmap.is_cuda and tuple(hmap.shape) == (plan.n_k, plan.n_x0) and hmap.is_contiguous()
    t = np.ascontiguousarray(tiles, dtype=np.int32)
    if cap is None:
        cap = max(1, 2 * int(sq_k) * int(sq_x0) * len(t))
    opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
    buf = (Candidate * max(1, cap))()
    counts = np.zeros(max(1, len(t)), dtype=np.int32)
    n = C.c_int32()
    _check(lib().fh_select_tiles(plan.handle, C.c_void_p(_ptr(hmap)), C.byref(opts), len(t), t.ctypes.data, buf,
                                 int(cap), counts.ctypes.data, C.byref(n), _stream(stream)), "fh_select_tiles")
    m = min(n.value, cap)
    recs = np.ctypeslib.as_array(buf)[:m].copy() if not as_dicts else [buf[i].as_dict() for i in range(m)]
    return recs, counts[:len(t)], int(n.value)


def fh_select_noalloc(plan: Plan, hmap, sq_k: int, sq_x0: int, min_dk: int = 3, cr_thr: float = -1e300,
                      col_lo: int = 0, col_hi: int = 0, cap: int = None, stream=None, as_dicts: bool = True):
    """fh_select through the allocation-free entry point (fixed scratch array in
    the library); same arguments and results."""
    assert hmap.is_cuda and tuple(hmap.shape) == (plan.n_k, plan.n_x0) and hmap.is_contiguous()
    if cap is None:
        cap = 2 * int(sq_k) * int(sq_x0)
    opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
    buf = (Candidate * max(1, cap))()
    n = C.c_int32()
    _check(lib().fh_select_noalloc(plan.handle, C.c_void_p(_ptr(hmap)), C.byref(opts), buf, int(cap), C.byref(n),
                                   _stream(stream)), "fh_select_noalloc")
    m = min(n.value, cap)
    if not as_dicts:
        import numpy as np
        return np.ctypeslib.as_array(buf)[:m].copy(), int(n.value)
    return [buf[i].as_dict() for i in range(m)], int(n.value)


def fh_hough_select(plan: Plan, row_ptr, bin_, out, sq_k: int, sq_x0: int, min_dk: int = 3,
                    cr_thr: float = -1e300, col_lo: int = 0, col_hi: int = 0, stream=None):
    """The Hough map (into `out`, int32 [n_k, n_x0] CUDA) and the selection of
    fh_select with these options in one pass, asynchronous on `stream`; the
    candidates come from fh_select_results(plan)."""
    import torch
    assert out.dtype == torch.int32 and out.is_contiguous() and tuple(out.shape) == (plan.n_k, plan.n_x0)
    if row_ptr.numel() != int(plan.info.n_fft) + 1:
        raise ValueError("row_ptr must have n_fft + 1 entries")
    pk = peaks_struct(row_ptr, bin_)
    opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
    _check(lib().fh_hough_select(plan.handle, C.byref(pk), C.c_void_p(_ptr(out)), C.byref(opts), _stream(stream)),
           "fh_hough_select")
    plan.sel_cap = 2 * int(sq_k) * int(sq_x0)
    return out


def fh_select_results(plan: Plan, cap: int = None, as_dicts: bool = True):
    """Candidates of the plan's last fh_hough_select, as fh_select returns them."""
    if cap is None:
        cap = getattr(plan, "sel_cap", 1)
    buf = (Candidate * max(1, cap))()
    n = C.c_int32()
    _check(lib().fh_select_results(plan.handle, buf, int(cap), C.byref(n)), "fh_select_results")
    m = min(n.value, cap)
    if not as_dicts:
        import numpy as np
        return np.ctypeslib.as_array(buf)[:m].copy(), int(n.value)
    return [buf[i].as_dict() for i in range(m)], int(n.value)


def fh_project(plan: Plan, row_ptr, bin_, f0, k, w: int = 40, guard: int = 2, stream=None):
    """Follow-up projection of the peakmap for each candidate (f0, k): float64
    CUDA tensors [n_cand].  Returns (hist int32 CUDA [n_cand, 2w+1], list of
    dicts y, mu, sigma, cr)."""
    import torch
    n = int(f0.numel())
    assert f0.is_cuda and k.is_cuda and f0.dtype == torch.float64 and k.dtype == torch.float64 and k.numel() == n
    assert f0.is_contiguous() and k.is_contiguous()
    hist = torch.empty((max(n, 1), 2 * int(w) + 1), dtype=torch.int32, device=f0.device)
    out = (Projection * max(n, 1))()
    pk = peaks_struct(row_ptr, bin_)
    _check(lib().fh_project(plan.handle, C.byref(pk), n, C.c_void_p(_ptr(f0)), C.c_void_p(_ptr(k)), int(w),
                            int(guard), C.c_void_p(_ptr(hist)), out,
                            _stream(stream)), "fh_project")
    return hist[:n], [{"y": out[i].y, "mu": out[i].mu, "sigma": out[i].sigma, "cr": out[i].cr,
                       "host_drift": out[i].host_drift} for i in range(n)]


def fh_coincide(a_off, a, b_off, b, max_d: float = 3.0, nm1=None, dt=None, cap: Optional[int] = None,
                stream=None):
    """Coincident pairs of two candidate lists (Sec. IV).  a, b: float64 CUDA
    tensors [n, 4] of (x0, k, dx0, dk); a_off, b_off: int32 CUDA tensors
    [n_seg + 1] delimiting each segment; nm1, dt: float64 CUDA tensors [n_seg]
    (move a's candidates along their lines by dt) or None.  Returns
    (pairs int32 [m, 2], dist float64 [m], total) with m = min(total, cap)."""
    import torch
    n_seg = int(a_off.numel()) - 1
    if n_seg < 0 or int(b_off.numel()) != n_seg + 1:
        raise ValueError("a_off and b_off need n_seg + 1 entries")
    for t, dt_ in ((a, torch.float64), (b, torch.float64), (a_off, torch.int32), (b_off, torch.int32)):
        assert t.is_cuda and t.dtype == dt_ and t.is_contiguous()
    if a.dim() != 2 or a.shape[1] != 4 or b.dim() != 2 or b.shape[1] != 4:
        raise ValueError("points are [n, 4] float64: x0, k, dx0, dk")
    na, nb = int(a.shape[0]), int(b.shape[0])
    dev = a.device
    count = torch.empty(1, dtype=torch.int32, device=dev)
    opt = lambda t: C.c_void_p(_ptr(t)) if t is not None else None

    def run(c):
        pairs = torch.empty((max(c, 1), 2), dtype=torch.int32, device=dev)
        dist = torch.empty(max(c, 1), dtype=torch.float64, device=dev)
        _check(lib().fh_coincide(n_seg, na, opt(a_off), opt(a) if na else None, nb, opt(b_off),
                                 opt(b) if nb else None, opt(nm1), opt(dt), float(max_d), C.c_void_p(_ptr(pairs)),
                                 C.c_void_p(_ptr(dist)), int(c), C.c_void_p(_ptr(count)), _stream(stream)),
               "fh_coincide")
        return pairs, dist, int(count.item())

    if cap is not None:
        pairs, dist, total = run(int(cap))
        m = min(total, int(cap))
        return pairs[:m], dist[:m], total
    pairs, dist, total = run(4 * max(na, nb, 1))
    if total > 4 * max(na, nb, 1):  # every pair wanted: run again with room for all
        pairs, dist, total = run(total)
    return pairs[:total], dist[:total], total


class Batch:
    """fh_batch_*: many maps in one persistent, graph-captured launch."""

    def __init__(self, plans: List[Plan], peaks: List[tuple], maps: List):
        m = len(plans)
        for p, (rp, _), x in zip(plans, peaks, maps):
            if rp.numel() != int(p.info.n_fft) + 1 or tuple(x.shape) != (p.n_k, p.n_x0):
                raise ValueError("peaks / map do not match the plan")
        self._keep = (plans, peaks, maps)
        self._plans = (C.c_void_p * m)(*[p.handle.value for p in plans])
        self._peaks = (Peaks * m)(*[peaks_struct(rp, b) for rp, b in peaks])
        self._maps = (C.c_void_p * m)(*[_ptr(x) for x in maps])
        h = C.c_void_p()
        _check(lib().fh_batch_create(m, self._plans, self._peaks, self._maps, C.byref(h)), "fh_batch_create")
        self.handle = h

    def select_tiles(self, req, sq_k: int, sq_x0: int, min_dk: int = 3, cr_thr: float = -1e300, col_lo: int = 0,
                     col_hi: int = 0, cap: int = None, stream=None):
        """fh_batch_select_tiles: the selection inside the (map index, tile index)
        pairs of req only: (candidate records, per-request counts, total)."""
        r = np.ascontiguousarray(req, dtype=np.int32).reshape(-1, 2)
        if cap is None:
            cap = max(1, 2 * int(sq_k) * int(sq_x0) * r.shape[0])
        opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
        buf = (Candidate * max(1, cap))()
        counts = np.zeros(max(1, r.shape[0]), dtype=np.int32)
        n = C.c_int32()
        _check(lib().fh_batch_select_tiles(self.handle, C.byref(opts), r.shape[0], r.ctypes.data, buf, int(cap),
                                           counts.ctypes.data, C.byref(n), _stream(stream)), "fh_batch_select_tiles")
        m = min(n.value, cap)
        return np.ctypeslib.as_array(buf)[:m].copy(), counts[:r.shape[0]], int(n.value)

    def launch(self, stream=None):
        _check(lib().fh_batch_launch(self.handle, _stream(stream)), "fh_batch_launch")

    def launch_plain(self, stream=None):
        _check(lib().fh_batch_launch_plain(self.handle, _stream(stream)), "fh_batch_launch_plain")

    def select(self, sq_k: int, sq_x0: int, min_dk: int = 3, cr_thr: float = -1e300, col_lo: int = 0,
               col_hi: int = 0, stream=None, as_dicts: bool = True):
        """fh_batch_select: the candidates of every map (after the last launch), as
        a list with one fh_select-style result per map."""
        m = len(self._keep[0])
        cap = 2 * int(sq_k) * int(sq_x0) * m
        opts = SelectOpts(int(sq_k), int(sq_x0), int(min_dk), int(col_lo), int(col_hi), float(cr_thr))
        buf = (Candidate * max(1, cap))()
        counts = (C.c_int32 * m)()
        n = C.c_int32()
        _check(lib().fh_batch_select(self.handle, C.byref(opts), buf, cap, counts, C.byref(n), _stream(stream)),
               "fh_batch_select")
        out, at = [], 0
        arr = np.ctypeslib.as_array(buf) if not as_dicts else None
        for i in range(m):
            c = int(counts[i])
            out.append([buf[j].as_dict() for j in range(at, at + c)] if as_dicts else arr[at:at + c].copy())
            at += c
        return out

    def destroy(self):
        if self.handle:
            lib().fh_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fh_hough_batched(plans: List[Plan], peaks: List[tuple], maps: List, stream=None):
    m = len(plans)
    P = (C.c_void_p * m)(*[p.handle.value for p in plans])
    K = (Peaks * m)(*[peaks_struct(rp, b) for rp, b in peaks])
    M = (C.c_void_p * m)(*[_ptr(x) for x in maps])
    _check(lib().fh_hough_batched(m, P, K, M, _stream(stream)), "fh_hough_batched")
    return maps


class CNN:
    """fh_cnn_*: the tile network (BF16 matrix-core kernels, FP32 master weights)."""

    def __init__(self, max_batch: int = 256):
        h = C.c_void_p()
        _check(lib().fh_cnn_create(int(max_batch), C.byref(h)), "fh_cnn_create")
        self.handle = h
        self.max_batch = int(max_batch)
        self.n_params = int(lib().fh_cnn_num_params())

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.n_params
        _check(lib().fh_cnn_set_params(self.handle, a.ctypes.data, a.size), "fh_cnn_set_params")

    def get_params(self):
        p = np.empty(self.n_params, dtype=np.float32)
        g = np.empty(self.n_params, dtype=np.float32)
        _check(lib().fh_cnn_get_params(self.handle, p.ctypes.data, g.ctypes.data, p.size), "fh_cnn_get_params")
        return p, g

    def set_grads(self, grads):
        """Replace the gradients the next step applies (host float array of n_params)."""
        a = np.ascontiguousarray(grads, dtype=np.float32)
        assert a.size == self.n_params
        _check(lib().fh_cnn_set_grads(self.handle, a.ctypes.data, a.size), "fh_cnn_set_grads")

    def get_state(self):
        """Adam's moments and step count: (m1, m2, steps)."""
        m1 = np.empty(self.n_params, dtype=np.float32)
        m2 = np.empty(self.n_params, dtype=np.float32)
        st = C.c_int64()
        _check(lib().fh_cnn_get_state(self.handle, m1.ctypes.data, m2.ctypes.data, m1.size, C.byref(st)),
               "fh_cnn_get_state")
        return m1, m2, int(st.value)

    def set_state(self, m1, m2, steps: int):
        a = np.ascontiguousarray(m1, dtype=np.float32)
        b = np.ascontiguousarray(m2, dtype=np.float32)
        assert a.size == b.size == self.n_params
        _check(lib().fh_cnn_set_state(self.handle, a.ctypes.data, b.ctypes.data, a.size, int(steps)),
               "fh_cnn_set_state")

    def activations(self, layer: int, batch: int):
        """BF16 activations of the last forward (layer 0: input, 1..4: conv outputs)
        as a float32 array [batch, 64, 64, C]."""
        ch = (1, 16, 32, 64, 64)[layer]
        raw = np.empty(batch * 64 * 64 * ch, dtype=np.uint16)
        _check(lib().fh_cnn_activations(self.handle, int(layer), raw.ctypes.data, raw.size), "fh_cnn_activations")
        return (raw.astype(np.uint32) << 16).view(np.float32).reshape(batch, 64, 64, ch)

    def forward(self, tiles, out=None, stream=None):
        """tiles: bfloat16 CUDA tensor [B, 64, 64]; returns float32 logits [B]."""
        import torch
        assert tiles.dtype == torch.bfloat16 and tiles.is_contiguous() and tuple(tiles.shape[1:]) == (64, 64)
        B = int(tiles.shape[0])
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device=tiles.device)
        _check(lib().fh_cnn_forward(self.handle, C.c_void_p(_ptr(tiles)), B, C.c_void_p(_ptr(out)),
                                    _stream(stream)), "fh_cnn_forward")
        return out

    def scores(self, tiles, out=None, stream=None):
        """fh_cnn_scores: the logits of fh_cnn_forward without keeping activations (no backward may follow)."""
        import torch
        assert tiles.dtype == torch.bfloat16 and tiles.is_contiguous() and tuple(tiles.shape[1:]) == (64, 64)
        B = int(tiles.shape[0])
        if out is None:
            out = torch.empty(B, dtype=torch.float32, device=tiles.device)
        _check(lib().fh_cnn_scores(self.handle, C.c_void_p(_ptr(tiles)), B, C.c_void_p(_ptr(out)), _stream(stream)),
               "fh_cnn_scores")
        return out

    def backward(self, labels, stream=None):
        """labels: float32 CUDA tensor [B] of the last forward; returns the loss tensor."""
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=labels.device)
        _check(lib().fh_cnn_backward(self.handle, C.c_void_p(_ptr(labels)), int(labels.numel()),
                                     C.c_void_p(_ptr(loss)), _stream(stream)), "fh_cnn_backward")
        return loss

    def step(self, lr: float, stream=None):
        _check(lib().fh_cnn_step(self.handle, float(lr), _stream(stream)), "fh_cnn_step")

    def destroy(self):
        if self.handle:
            lib().fh_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fh_tiles(hmap, origins, stream=None):
    """Normalised BF16 tiles [n, 64, 64] of an int32 CUDA map at origins (int32 CUDA [n, 2])."""
    import torch
    n_k, n_x0 = hmap.shape
    n = int(origins.shape[0])
    tiles = torch.empty((n, 64, 64), dtype=torch.bfloat16, device=hmap.device)
    mean = torch.empty(n_k, dtype=torch.float32, device=hmap.device)
    istd = torch.empty(n_k, dtype=torch.float32, device=hmap.device)
    _check(lib().fh_tiles(C.c_void_p(_ptr(hmap)), n_k, n_x0, C.c_void_p(_ptr(origins)), n, C.c_void_p(_ptr(tiles)),
                          C.c_void_p(_ptr(mean)), C.c_void_p(_ptr(istd)), _stream(stream)), "fh_tiles")
    return tiles


def fh_batch_propose(net: CNN, batch: Batch, n_top: Sequence[int], stream=None):
    """(scores CUDA float32 [all tiles, map after map], list of each map's best
    tile indices)."""
    import torch
    plans = batch._keep[0]
    n_tiles = [((p.n_k + 63) // 64) * ((p.n_x0 + 63) // 64) for p in plans]
    scores = torch.empty(max(1, sum(n_tiles)), dtype=torch.float32, device=batch._keep[2][0].device)
    nt = (C.c_int32 * len(plans))(*[int(x) for x in n_top])
    ids = np.zeros(max(1, sum(int(x) for x in n_top)), dtype=np.int32)
    _check(lib().fh_batch_propose(net.handle, batch.handle, C.c_void_p(_ptr(scores)), nt, ids.ctypes.data,
                                  _stream(stream)), "fh_batch_propose")
    out, at = [], 0
    for x in n_top:
        out.append([int(i) for i in ids[at:at + int(x)]])
        at += int(x)
    return scores[:sum(n_tiles)], out


def fh_propose(net: CNN, plan: Plan, hmap, n_top: int, stream=None):
    """(scores [n_tiles] CUDA float32, best tile indices as a list)."""
    import torch
    ta, tb = (plan.n_k + 63) // 64, (plan.n_x0 + 63) // 64
    scores = torch.empty(ta * tb, dtype=torch.float32, device=hmap.device)
    ids = np.zeros(max(1, n_top), dtype=np.int32)
    _check(lib().fh_propose(net.handle, plan.handle, C.c_void_p(_ptr(hmap)), C.c_void_p(_ptr(scores)), int(n_top),
                            ids.ctypes.data, _stream(stream)), "fh_propose")
    return scores, [int(i) for i in ids[:n_top]]
