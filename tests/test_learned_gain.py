"""What the trained tile CNN gains over the plain selection alone (GPU).  At
a false-alarm probability of 1e-3 per map, both pipelines' thresholds set on
10^4 noise-only maps, the learned pipeline (the network's best tile of 12,
re-checked by the selection with the tile's own statistics) must reach the
plain selection's detection efficiency within 2%, resolved: on 2000 injected
maps per amplitude, compared map by map, the difference must exceed -2% by
two standard errors.  An untrained network does not get there."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1810_09784_amd",
                       "trained", "tile_cnn.npy")


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    fh.lib()
    return torch.device("cuda:0")


def test_trained_proposer_within_two_percent_at_fap_1e3(dev):
    from paper_1810_09784_amd import fh, learn
    net = fh.CNN(max_batch=256)
    net.set_params(np.load(WEIGHTS))
    # fresh seeds: neither the training nor the stored evaluation used them
    res = learn.evaluate(dev, net, [0.4, 0.7], n_noise=10000, n_per_amp=2000, seed=9100, fap=1e-3)
    assert res["tiles_touched_frac"] <= 0.10
    # the thresholds hold the false-alarm probability on their 10^4 noise maps
    # (at most 1e-3 by construction; ties could only lower it)
    for key in ("fap_plain", "fap_learned"):
        assert 0.5e-3 <= res[key] <= 1e-3, res
    for pt in res["curve"]:
        assert pt["n"] == 2000
        assert 0.1 < pt["eff_plain"] < 0.9, pt  # the amplitudes where efficiency can differ
        assert pt["diff"] >= -0.02 + 2.0 * pt["se_diff"], pt
    net.destroy()


def test_untrained_network_loses_the_signals(dev):
    from paper_1810_09784_amd import fh, learn
    from oracle import cnn as N
    net = fh.CNN(max_batch=256)
    net.set_params(N.init_params(np.random.default_rng(3)))
    res = learn.evaluate(dev, net, [1.0], n_noise=1000, n_per_amp=400, seed=9200, fap=1e-2)
    pt = res["curve"][0]
    assert pt["eff_learned"] < 0.6 * pt["eff_plain"], res
    net.destroy()
