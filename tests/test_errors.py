"""Error paths forced from the host (GPU): allocation failures (FH_FAKE_OOM),
a failed graph instantiation (FH_FAKE_DEVICE_ERROR=graph), a misaligned bin
array, and the bad-peak counter in every way the library counts it.  Every
kernel that runs here exits normally; the failures are injected on the host
before anything is launched."""
import ctypes as C

import numpy as np
import pytest

from paper_1810_09784_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    fh.lib()
    return torch.device("cuda:0")


def _small(rng):
    return S.cfg_tiny(rng, n_fft=80, n_f=60, n_k=12, n=4.0, tfft=2.0, f_min=400.0, kscale=0.2)


def _on_dev(pm, dev):
    import torch
    return torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev)


def test_fake_oom_every_allocating_entry_point(dev, monkeypatch):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(1)
    spec = _small(rng)
    pm = S.make_peakmap(spec)
    rp, bn = _on_dev(pm, dev)
    plan = fh.Plan.from_spec(spec)  # made before the hook is set
    H = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    fh.fh_hough(plan, rp, bn, H)  # plan-owned scratch: no allocation here
    monkeypatch.setenv("FH_FAKE_OOM", "1")
    with pytest.raises(fh.FHError) as e:
        fh.Plan.from_spec(spec)
    assert e.value.status == fh.FH_ENOMEM
    with pytest.raises(fh.FHError) as e:  # the selection scratch is allocated on first use
        fh.fh_select(plan, H, 3, 3, 3)
    assert e.value.status == fh.FH_ENOMEM
    with pytest.raises(fh.FHError) as e:
        fh.CNN(max_batch=2)
    assert e.value.status == fh.FH_ENOMEM
    with pytest.raises(fh.FHError) as e:
        fh.Batch([plan], [(rp, bn)], [H])
    assert e.value.status == fh.FH_ENOMEM
    # fh_hough itself allocates nothing: it still works under the hook
    fh.fh_hough(plan, rp, bn, H)
    monkeypatch.delenv("FH_FAKE_OOM")
    fh.fh_select(plan, H, 3, 3, 3)  # and the selection recovers once allocation works again


def test_fake_graph_failure_writes_nothing(dev, monkeypatch):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(2)
    specs = [_small(rng), _small(rng)]
    plans, peaks, maps = [], [], []
    for s in specs:
        pm = S.make_peakmap(s)
        plans.append(fh.Plan.from_spec(s))
        peaks.append(_on_dev(pm, dev))
        maps.append(torch.full((plans[-1].n_k, plans[-1].n_x0), -7, dtype=torch.int32, device=dev))
    monkeypatch.setenv("FH_FAKE_DEVICE_ERROR", "graph")
    with pytest.raises(fh.FHError) as e:
        fh.Batch(plans, peaks, maps)
    assert e.value.status == fh.FH_EDEVICE
    torch.cuda.synchronize()
    assert all(bool((m == -7).all()) for m in maps)  # nothing ran
    monkeypatch.delenv("FH_FAKE_DEVICE_ERROR")
    b = fh.Batch(plans, peaks, maps)
    b.launch()
    torch.cuda.synchronize()
    assert all(bool((m >= 0).all()) for m in maps)
    b.destroy()


def test_misaligned_bins_rejected(dev):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(3)
    spec = _small(rng)
    pm = S.make_peakmap(spec)
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    padded = torch.from_numpy(np.concatenate([[0], pm.bin]).astype(np.int32)).to(dev)
    bn = padded[1:]  # 4 bytes past a 16-byte boundary
    assert bn.data_ptr() % 16 == 4
    plan = fh.Plan.from_spec(spec)
    H = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    for call in (lambda: fh.fh_hough(plan, rp, bn, H), lambda: fh.fh_hough_select(plan, rp, bn, H, 3, 3, 3),
                 lambda: fh.Batch([plan], [(rp, bn)], [H])):
        with pytest.raises(fh.FHError) as e:
            call()
        assert e.value.status == fh.FH_EINVAL
    torch.cuda.synchronize()
    assert bool((H == -7).all())


def _bad_peakmap(rng, spec):
    """A peakmap with every kind of bad peak: out-of-band bins (below, above,
    one that also breaks the order), a repeated bin, a reversed FFT."""
    pm = S.make_peakmap(spec)
    rows = [list(pm.bin[pm.row_ptr[i]:pm.row_ptr[i + 1]]) for i in range(spec.n_fft)]
    full = [i for i in range(spec.n_fft) if len(rows[i]) >= 4]
    rows[full[0]] = [-5] + rows[full[0]]                          # below the band, first
    rows[full[1]] = rows[full[1]] + [spec.n_f + 2]                # above the band, last
    rows[full[2]] = rows[full[2]][:2] + [-1] + rows[full[2]][2:]  # below the band and not ascending
    rows[full[3]] = rows[full[3]][:2] + [rows[full[3]][1]] + rows[full[3]][2:]  # a repeated bin
    rows[full[4]] = rows[full[4]][::-1]                           # reversed
    bad = 0
    for r in rows:
        for q, j in enumerate(r):
            bad += (not 0 <= j < spec.n_f) or (q > 0 and j <= r[q - 1])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    return S.Peakmap(rp, np.concatenate([np.asarray(r, dtype=np.int32) for r in rows]), spec.n_fft, spec.n_f), bad


@pytest.mark.parametrize("n_f,tile", [
    (60, dict(mode=1, rows=4, cols=64, threads=256, tsplit=1)),      # whole-FFT tiles count
    (60, dict(mode=1, rows=3, cols=30, threads=512, tsplit=3)),      # the counting tile split in FFT ranges
    (3000, dict(mode=2, rows=1, cols=512, threads=256, tsplit=2)),   # rank build in LDS
    (17000, dict(mode=2, rows=1, cols=4096, threads=256, tsplit=1)),  # rank build by bisection
])
def test_bad_peaks_counted_once(dev, oracle, n_f, tile):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(7 + n_f)
    spec = S.cfg_tiny(rng, n_fft=40, n_f=n_f, n_k=6, n=3.0, tfft=4.0, f_min=300.0, kscale=0.05)
    pm, bad = _bad_peakmap(rng, spec)
    plan = fh.Plan.from_spec(spec, tile=tile)
    assert plan.tile["mode"] == tile["mode"]
    rp, bn = _on_dev(pm, dev)
    H = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    fh.fh_hough(plan, rp, bn, H)
    errs = fh.fh_device_errors(plan)
    if n_f > 16384:
        assert errs >= 5  # one per bad FFT at least (bisection path)
    else:
        assert errs == bad, (errs, bad)
    if tile["mode"] == 1:  # whole-FFT counting does not depend on the order of an FFT's peaks
        ref = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin)
        assert np.array_equal(H.cpu().numpy(), ref)
