"""The C ABI: the library loads, exports every symbol the header declares, and
rejects invalid map descriptions on the host before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1810_09784_amd import fh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(fh_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = fh.lib()
    names = declared_symbols()
    assert {"fh_plan", "fh_hough", "fh_hough_batched"} <= names
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(fh.SIGNATURES) == names


def _plan_status(**kw):
    base = dict(n=3.0, tfft=2.0, f_min=100.0, f_max=150.0, n_fft=10, k=[0.0, 1e-9], t=None, x0_min=0.0, dx0=0.0,
                n_x0=0)
    base.update(kw)
    k = np.ascontiguousarray(base["k"], dtype=np.float64)
    t = None if base["t"] is None else np.ascontiguousarray(base["t"], dtype=np.float64)
    dp = C.POINTER(C.c_double)
    d = fh.MapDesc(base["n"], base["tfft"], base["f_min"], base["f_max"], base["n_fft"],
                   dp() if t is None else t.ctypes.data_as(dp), len(k), k.ctypes.data_as(dp), base["x0_min"],
                   base["dx0"], base["n_x0"])
    h = C.c_void_p()
    st = fh.lib().fh_plan(C.byref(d), None, C.byref(h))
    if st == 0:
        fh.lib().fh_plan_destroy(h)
    return st


@pytest.mark.parametrize("kw,expect", [
    (dict(n=1.0), fh.FH_EINVAL),
    (dict(n=0.5), fh.FH_EINVAL),
    (dict(n=float("nan")), fh.FH_EINVAL),
    (dict(tfft=0.0), fh.FH_EINVAL),
    (dict(f_min=150.0, f_max=100.0), fh.FH_EINVAL),
    (dict(f_min=0.0), fh.FH_EINVAL),
    (dict(f_max=150.3), fh.FH_EINVAL),                  # band not a whole number of bins
    (dict(k=[1e-9, 0.0]), fh.FH_EINVAL),                # k not ascending
    (dict(k=[-1e-9, 0.0]), fh.FH_EINVAL),               # k < 0
    (dict(k=[0.0, float("inf")]), fh.FH_EINVAL),
    (dict(n_fft=0), fh.FH_EINVAL),
    (dict(t=[0.0] * 9 + [-1.0]), fh.FH_EINVAL),         # times not ascending
    (dict(dx0=-1.0), fh.FH_EINVAL),
    (dict(n_x0=-3), fh.FH_EINVAL),
    (dict(n_x0=2**30, k=[0.0, 1e-9, 2e-9]), fh.FH_ERANGE),  # n_k * n_x0 >= 2^31
    (dict(f_min=1.0, f_max=1.0 + 2**25), fh.FH_ERANGE),
])
def test_invalid_descriptions_rejected_on_host(kw, expect):
    assert _plan_status(**kw) == expect


def test_null_arguments():
    L = fh.lib()
    h = C.c_void_p()
    assert L.fh_plan(None, None, C.byref(h)) == fh.FH_EINVAL
    assert L.fh_hough(None, None, None, None) == fh.FH_EINVAL
    assert L.fh_batch_create(0, None, None, None, C.byref(h)) == fh.FH_EINVAL
    assert fh.status_str(fh.FH_ERANGE) == "size out of range"
    assert b"gfx950" in L.fh_version()


def _peaks(row_ptr_addr, bin_addr, n):
    return fh.Peaks(C.c_void_p(row_ptr_addr), C.c_void_p(bin_addr), n)


def test_peaks_validated_on_host():
    # fh_peaks_validate reads no memory: host addresses stand in for device ones
    L = fh.lib()
    buf = np.zeros(64, dtype=np.int32)
    a = buf.ctypes.data
    base = a + (-a) % 16  # a 16-byte aligned address inside the buffer
    assert L.fh_peaks_validate(None) == fh.FH_EINVAL
    assert L.fh_peaks_validate(C.byref(_peaks(base, base, 10))) == fh.FH_OK
    assert L.fh_peaks_validate(C.byref(_peaks(base, base + 4, 10))) == fh.FH_EINVAL   # bin not 16-byte aligned
    assert L.fh_peaks_validate(C.byref(_peaks(base, base + 8, 10))) == fh.FH_EINVAL
    assert L.fh_peaks_validate(C.byref(_peaks(0, base, 10))) == fh.FH_EINVAL          # no row_ptr
    assert L.fh_peaks_validate(C.byref(_peaks(base, 0, 10))) == fh.FH_EINVAL          # no bins for 10 peaks
    assert L.fh_peaks_validate(C.byref(_peaks(base, 0, 0))) == fh.FH_OK               # an empty peakmap
    assert L.fh_peaks_validate(C.byref(_peaks(base, base, -1))) == fh.FH_EINVAL
    assert L.fh_peaks_validate(C.byref(_peaks(base, base, 2 ** 31))) == fh.FH_EINVAL
    # fh_hough rejects the same before using its plan
    assert L.fh_hough(None, C.byref(_peaks(base, base + 4, 10)), C.c_void_p(base), None) == fh.FH_EINVAL


def test_fake_oom_fails_the_plan_before_any_device_memory(monkeypatch):
    monkeypatch.setenv("FH_FAKE_OOM", "1")
    k = np.ascontiguousarray([0.0, 1e-9], dtype=np.float64)
    dp = C.POINTER(C.c_double)
    d = fh.MapDesc(3.0, 2.0, 100.0, 150.0, 10, dp(), 2, k.ctypes.data_as(dp), 0.0, 0.0, 0)
    h = C.c_void_p()
    assert fh.lib().fh_plan(C.byref(d), None, C.byref(h)) == fh.FH_ENOMEM
    assert not h.value
