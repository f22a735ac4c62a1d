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
    # every stored entry is a shape the library accepts for its map (or, for a
    # batch, one shape per map, all with the same work-group size)
    for k, e in tune._load().items():
        tiles = e["tiles"] if k.startswith("batch") else [e["tile"]]
        for t in tiles:
            assert set(t) >= {"rows", "cols", "threads", "mode", "tsplit"}
        assert len({t["threads"] for t in tiles}) == 1
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


def test_batch_candidates_and_tiles():
    cands = tune.batch_candidates()
    assert cands[0] is None and len(cands) == 1 + len(tune.BATCH_THREADS) * len(tune.BATCH_TILE_KB) * \
        len(tune.BATCH_TSPLIT)
    for n_x0, n_k in ((69, 703), (850, 300), (8500, 40), (300, 3)):
        for kb in tune.BATCH_TILE_KB:
            t = tune.batch_tile(n_x0, n_k, 512, kb, 16)
            assert t["mode"] == 1 and t["cols"] == min(n_x0, 8192) and t["threads"] == 512
            r = t["rows"]
            assert 1 <= r <= min(64, n_k) and (r & (r - 1) == 0 or r == n_k)
            pitch = (t["cols"] + 4) // 4 * 4
            assert r == 1 or r == min(64, n_k) or r * pitch * 4 <= kb * 1024 < 2 * r * pitch * 4
    specs = S.cfg_batched()[:3]
    k = tune.batch_key(specs, [10, 20, 30])
    assert k == tune.batch_key(S.cfg_batched()[:3], [10, 20, 30]) and k != tune.batch_key(specs, [10, 20, 10 ** 7])
    assert tune.lookup_batch(specs, [1, 2, 3]) is None


@pytest.mark.gpu
def test_autotune_batch_small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(8)
    specs = [S.cfg_tiny(rng, n_fft=200 + 50 * i, n_f=40 + 30 * i, n_k=20 + 7 * i, n=3.0 + i, tfft=2.0,
                        f_min=300.0 + 50 * i) for i in range(4)]
    pms = [S.make_peakmap(s) for s in specs]
    cands = [None, dict(threads=256, tile_kb=12, tsplit=16), dict(threads=1024, tile_kb=40, tsplit=64)]
    e = tune.autotune_batch(specs, pms, torch.device("cuda:0"), reps=2, save=False, candidates=cands)
    assert e["n_candidates"] == 3 and e["ms"] > 0 and len(e["tiles"]) == 4  # every candidate: the same maps
