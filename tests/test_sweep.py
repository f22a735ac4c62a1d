"""A reduced full-sweep run (same code path as the 990-map workload): every
map exact against the oracle, and the evaluation runs end to end."""
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


def test_reduced_sweep_exact_and_evaluated(dev, oracle):
    import os
    import torch
    from paper_1810_09784_amd import fh, sweep
    sw = sweep.Sweep(dev, seed=9, n_values=(2.5, 5.0, 7.0), tffts=(4.0, 8.0), n_bands=2, t_obs=1.2e4, n_k=64,
                     n_inj=6, amp_lo=3.0, amp_hi=6.0)
    assert len(sw.maps) == 2 * 2 * 3
    sw.batch.launch()
    torch.cuda.synchronize()
    for m in sw.maps:
        rp, bn = sw.peakmaps[(m["band"], m["ti"])]
        d = oracle.Desc(m["n"], m["tfft"], m["f_min"], m["f_max"], m["n_fft"], m["k"])
        ref = oracle.hough(d, rp.cpu().numpy(), bn.cpu().numpy())
        assert np.array_equal(m["hmap"].cpu().numpy(), ref), (m["band"], m["tfft"], m["n"])
    net = fh.CNN(max_batch=64)
    net.set_params(np.load(os.path.join(os.path.dirname(fh.__file__), "trained", "tile_cnn.npy")))
    ev = sweep.evaluate(sw, net, sq=(8, 8))
    assert ev["tiles"] > 0 and len(ev["curves"]) == 3
    for c in ev["curves"]:
        assert 0.0 <= c["eff_learned"] <= c["eff_plain"] <= 1.0
    assert ev["curves"][0]["eff_plain"] > 0.5
    sw.destroy()


def test_reduced_sweep_on_the_paper_k_grids(dev, oracle):
    # the same run with each map on the geometric k grid of its T_FFT level
    # (fdot in [1/(2 T_FFT)^2, 1/T_FFT^2]); injections on rows of those grids
    import torch
    from paper_1810_09784_amd import grids, sweep
    sw = sweep.Sweep(dev, seed=19, n_values=(2.5, 5.0), tffts=(4.0, 8.0), n_bands=2, t_obs=1.2e4, n_inj=6,
                     amp_lo=3.0, amp_hi=6.0, k_layout="paper")
    for m in sw.maps:
        ks, _ = grids.k_grid(m["n"], m["tfft"], m["f_min"], m["f_max"], 1.0 / (2 * m["tfft"]) ** 2, 1.0 / m["tfft"] ** 2)
        assert np.array_equal(m["k"], ks)
    sw.batch.launch()
    torch.cuda.synchronize()
    for m in sw.maps:
        rp, bn = sw.peakmaps[(m["band"], m["ti"])]
        d = oracle.Desc(m["n"], m["tfft"], m["f_min"], m["f_max"], m["n_fft"], m["k"])
        ref = oracle.hough(d, rp.cpu().numpy(), bn.cpu().numpy())
        assert np.array_equal(m["hmap"].cpu().numpy(), ref), (m["band"], m["tfft"], m["n"])
    ev = sweep.evaluate(sw, None, sq=(8, 8))
    assert ev["curves"][0]["eff_plain"] > 0.5
    sw.destroy()


def test_reduced_sweep_at_fixed_fap(dev, oracle):
    # noise-only maps' largest candidate CR (plain pipeline) matches the
    # oracle's selection on the oracle's maps; thresholds from those maxima keep
    # the false-alarm fraction at or under each requested probability and
    # rise as it falls, and efficiencies fall with them
    import os
    from oracle import select as oracle_select
    from paper_1810_09784_amd import fh, sweep
    kw = dict(n_values=(2.5, 5.0), tffts=(4.0, 8.0), n_bands=2, t_obs=1.2e4, n_k=64)
    net = fh.CNN(max_batch=64)
    net.set_params(np.load(os.path.join(os.path.dirname(fh.__file__), "trained", "tile_cnn.npy")))
    nsw = sweep.Sweep(dev, seed=31, n_inj=0, **kw)
    mx = sweep.map_maxima(nsw, net, sq=(8, 8))
    for mi, m in enumerate(nsw.maps):
        rp, bn = nsw.peakmaps[(m["band"], m["ti"])]
        d = oracle.Desc(m["n"], m["tfft"], m["f_min"], m["f_max"], m["n_fft"], m["k"])
        ref = oracle.hough(d, rp.cpu().numpy(), bn.cpu().numpy())
        _, x0m, dx, _ = oracle.grid(d)
        rc = oracle_select.select(ref, m["k"], x0m, dx, m["n"], 8, 8, 3)
        want = max((c["cr"] for c in rc), default=-np.inf)
        assert mx[mi, 0] == pytest.approx(want, rel=1e-12, abs=1e-12), mi
        assert mx[mi, 1] <= mx[mi, 0]
    nsw.destroy()
    sw = sweep.Sweep(dev, seed=32, n_inj=8, amp_lo=2.0, amp_hi=6.0, **kw)
    faps = [0.5, 0.25, 0.125]
    res = sweep.evaluate_at_fap(dev, net, faps, 3, 33, sw=sw, sq=(8, 8), **kw)
    sw.destroy()
    assert [r["fap_per_map"] for r in res] == faps
    for r in res:
        assert r["noise_maps"] == 3 * len(sw.maps)
        assert r["fap_plain"] <= r["fap_per_map"] and r["fap_learned"] <= r["fap_per_map"]
        assert 0.0 <= r["eff_plain"] <= 1.0 and 0.0 <= r["eff_learned"] <= 1.0
        assert sum(b["n"] for b in r["by_amp"]) <= r["injections"] == 8
    for a, b in zip(res[:-1], res[1:]):
        assert b["thr_plain"] >= a["thr_plain"] and b["thr_learned"] >= a["thr_learned"]
        assert b["eff_plain"] <= a["eff_plain"] and b["eff_learned"] <= a["eff_learned"]


def test_resumable_sweep_continues_after_a_crash(dev, tmp_path):
    # a reduced sweep run through the per-map checkpoint, interrupted after its
    # first group of maps (and with a torn record at the end of the file), then
    # resumed: the result equals an uninterrupted run, and the maps done before
    # the crash are not computed again
    from paper_1810_09784_amd import sweep
    kw = dict(n_values=(2.0, 4.5), tffts=(2.0, 8.0), n_bands=2, t_obs=20000.0, n_k=48, n_inj=4, seed=17)
    full = str(tmp_path / "full.jsonl")
    assert sweep.run_resumable(dev, full, cr_thr=3.0, **kw) == 8

    class Crash(Exception):
        pass

    def crash(b, ti):
        raise Crash()

    part = str(tmp_path / "part.jsonl")
    try:
        sweep.run_resumable(dev, part, cr_thr=3.0, after_group=crash, **kw)
    except Crash:
        pass
    with open(part, "a") as f:
        f.write('{"key": [4.5, 8.0')
    assert sweep.run_resumable(dev, part, cr_thr=3.0, **kw) == 6  # the first group's 2 maps were done
    a = sweep.Checkpoint(full).done
    b = sweep.Checkpoint(part).done
    assert a.keys() == b.keys() and len(a) == 8
    for k in a:
        assert a[k] == b[k], k
    assert any(r["candidates"] for r in a.values())
