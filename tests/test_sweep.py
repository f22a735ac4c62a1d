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
