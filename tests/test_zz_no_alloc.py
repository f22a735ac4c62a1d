"""fh_select_noalloc (the selection on the library's fixed scratch array)
against fh_select on the same maps: two calls in a row, the second on a smaller
map, several host-finish chunks, and the size limit."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    fh.lib()
    return torch.device("cuda:0")


def _map(dev, spec):
    import torch
    from paper_1810_09784_amd import fh, synth
    pm = synth.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    H = fh.fh_hough(plan, torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev))
    return plan, H, pm


def _same(a, b):
    assert b[1] == a[1]
    ra, rb = a[0], b[0]
    assert len(ra) == len(rb)
    for x, y in zip(ra, rb):
        assert x == y  # every field, the binary64 ones bit for bit


def test_noalloc_equals_fh_select_twice(dev):
    from paper_1810_09784_amd import fh, synth
    rng = np.random.default_rng(41)
    # a wider map first: 16 x 32 = 512 squares, two chunks of the host finish
    big = synth.cfg_tiny(rng, n_fft=3000, n_f=600, n_k=300, n=4.0, tfft=2.0, f_min=300.0)
    plan_b, H_b, _ = _map(dev, big)
    ref = fh.fh_select(plan_b, H_b, 16, 32, 3)
    got = fh.fh_select_noalloc(plan_b, H_b, 16, 32, 3)
    _same(ref, got)
    # then a smaller map with fewer squares: nothing of the first call may leak in
    small = synth.cfg_single_small()
    small.n_fft = 2400
    plan_s, H_s, pm = _map(dev, small)
    ref = fh.fh_select(plan_s, H_s, 5, 5, 3, cr_thr=2.0)
    got = fh.fh_select_noalloc(plan_s, H_s, 5, 5, 3, cr_thr=2.0)
    _same(ref, got)
    # and against the oracle's selection of the oracle's map
    from oracle import hough as oracle
    from oracle import select as oracle_select
    d = oracle.Desc.from_spec(small)
    omap = oracle.hough(d, pm.row_ptr, pm.bin)
    assert np.array_equal(H_s.cpu().numpy(), omap)
    _, x0m, dx, _ = oracle.grid(d)
    oc = oracle_select.select(omap, small.k, x0m, dx, small.n, 5, 5, 3, cr_thr=2.0)
    assert len(oc) == got[1]
    for c, r in zip(got[0], oc):
        assert (c["row"], c["col"], c["count"], c["square"], c["second"], c["cr"]) == \
               (r["row"], r["col"], r["count"], r["square"], r["second"], r["cr"])
    # a short output buffer: the same first records and the same total
    _same(fh.fh_select(plan_s, H_s, 5, 5, 3, cap=7), fh.fh_select_noalloc(plan_s, H_s, 5, 5, 3, cap=7))


def test_noalloc_size_limit(dev):
    import torch
    from paper_1810_09784_amd import fh, synth
    spec = synth.cfg_single_large()
    spec.n_fft = 16
    plan = fh.Plan.from_spec(spec)  # 1024 x 84000
    H = torch.randint(0, 1000, (plan.n_k, plan.n_x0), dtype=torch.int32, device=dev, generator=torch.Generator(
        device=dev).manual_seed(7))
    # 1024 x 256 x 3 words of row partials exceed the 2^19-word array: rejected,
    # nothing written
    opts = fh.SelectOpts(5, 256, 3, 0, 0, -1e300)
    buf = (fh.Candidate * 4)()
    n = C.c_int32(-123)
    st = fh.lib().fh_select_noalloc(plan.handle, C.c_void_p(H.data_ptr()), C.byref(opts), buf, 4, C.byref(n),
                                    fh._stream(None))
    assert st == fh.FH_ERANGE and n.value == -123
    # just inside the limit (1024 x 160 x 3 + 6 x 5 x 160 words) it equals fh_select
    assert 1024 * 160 * 3 + 6 * 5 * 160 <= 1 << 19
    _same(fh.fh_select(plan, H, 5, 160, 3), fh.fh_select_noalloc(plan, H, 5, 160, 3))
