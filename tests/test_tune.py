"""The tile-shape autotuner: its candidate shapes, cache keys and lookups
(CPU), and a tuning run on a small map in both timing arrangements (GPU),
in which every candidate must produce the same map."""
import numpy as np
import pytest

from paper_1810_09784_amd import synth as S
from paper_1810_09784_amd import tune


def test_candidates_are_valid_shapes():
    for n_x0, n_k, n_fft in ((300, 64, 5000), (84000, 1024, 43200), (9000, 7, 3)):
        cs = tune.candidates(n_x0, n_k, n_fft)
        assert cs[0] is None  # the library's own choice is always a candidate
        for c in cs[1:]:
            assert c["mode"] in (1, 2) and c["threads"] in (256, 512, 1024)
            assert 1 <= c["rows"] <= n_k and c["tsplit"] >= 1  # tsplit caps the pieces of a tile
            assert 1 <= c["cols"] <= n_x0
            if c["mode"] == 1:
                assert c["cols"] == n_x0  # whole-FFT tiles span the map's columns
            else:
                assert c["cols"] <= 40000


def test_cache_keys_and_lookup():
    s = S.cfg_single_small()
    k1 = tune.key(s, 18608)
    assert k1 == tune.key(S.cfg_single_small(), 18608)
    assert k1 != tune.key(s, 18609 * 2)  # the peak density is part of the key
    assert tune.lookup(S.cfg_tiny(np.random.default_rng(0), 7, 11, 3), 5) is None
    # every stored entry is a shape the library accepts for its map
    for e in tune._load().values():
        assert set(e["tile"]) >= {"rows", "cols", "threads", "mode", "tsplit"}
        assert e["ms"] > 0 and e["n_candidates"] >= 1


@pytest.mark.gpu
@pytest.mark.parametrize("streams,select", [(1, None), (2, None), (2, (3, 3, 3))])
def test_autotune_small_map(streams, select):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(7)
    spec = S.cfg_tiny(rng, n_fft=300, n_f=120, n_k=40, n=3.0, tfft=2.0, f_min=300.0)
    pm = S.make_peakmap(spec)
    e = tune.autotune(spec, pm, torch.device("cuda:0"), reps=2, save=False, streams=streams, select=select)
    assert e["n_candidates"] >= 2 and e["ms"] > 0 and e["streams"] == streams
    assert e["timed"] == ("fh_hough" if select is None else "fh_hough_select(3, 3, 3)")
    assert set(e["tile"]) >= {"rows", "cols", "threads", "mode", "tsplit"}
