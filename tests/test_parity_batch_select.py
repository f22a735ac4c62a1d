"""fh_batch_select (one row pass and one square reduction over every map of a
batch) against the oracle selection and against per-map fh_select, on the 48
uneven maps of the batched workload."""
import numpy as np
import pytest

from paper_1810_09784_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch48():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_09784_amd import fh
    dev = torch.device("cuda:0")
    specs = S.cfg_batched()
    plans, peaks, maps, pms = [], [], [], []
    for s in specs:
        pm = S.make_peakmap(s)
        pl = fh.Plan.from_spec(s)
        plans.append(pl)
        pms.append(pm)
        peaks.append((torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev)))
        maps.append(torch.empty((pl.n_k, pl.n_x0), dtype=torch.int32, device=dev))
    batch = fh.Batch(plans, peaks, maps)
    batch.launch()
    torch.cuda.synchronize()
    yield specs, pms, plans, maps, batch
    batch.destroy()


def _same(got, ref):
    assert len(got) == len(ref), (len(got), len(ref))
    for g, r in zip(got, ref):
        for key in ("row", "col", "count", "square", "second"):
            assert g[key] == r[key], (key, g, r)
        for key in ("cr", "mu", "sigma", "x0", "k", "f0", "fdot0"):
            assert g[key] == r[key] or (np.isnan(g[key]) and np.isnan(r[key])), (key, g[key], r[key])


@pytest.mark.parametrize("sq,min_dk,thr,cols", [((8, 8), 3, -1e300, (0, 0)), ((3, 5), 2, 1.5, (0, 0)),
                                                ((16, 1), 0, -1e300, (2, 0)), ((1, 30), 5, 0.0, (10, 60))])
def test_batch_select_equals_per_map(batch48, sq, min_dk, thr, cols):
    from paper_1810_09784_amd import fh
    specs, pms, plans, maps, batch = batch48
    got = batch.select(sq[0], sq[1], min_dk, thr, col_lo=cols[0], col_hi=cols[1])
    assert len(got) == len(plans)
    for pl, H, g in zip(plans, maps, got):
        ref, n = fh.fh_select(pl, H, sq[0], sq[1], min_dk, thr, col_lo=cols[0], col_hi=cols[1])
        assert n == len(g)
        _same(g, ref)


def test_batch_select_against_oracle(batch48, oracle):
    from oracle import select as OS
    specs, pms, plans, maps, batch = batch48
    got = batch.select(6, 4, 3)
    for i in (0, 17, 47):
        d = oracle.Desc.from_spec(specs[i])
        ref_map = oracle.hough(d, pms[i].row_ptr, pms[i].bin)
        assert np.array_equal(maps[i].cpu().numpy(), ref_map)
        nf, x0m, dx, nx = oracle.grid(d)
        _same(got[i], OS.select(ref_map, specs[i].k, x0m, dx, specs[i].n, 6, 4, 3))


def test_batch_select_rejects_options_invalid_for_a_map(batch48):
    from paper_1810_09784_amd import fh
    specs, pms, plans, maps, batch = batch48
    n_k_min = min(p.n_k for p in plans)
    with pytest.raises(fh.FHError):
        batch.select(n_k_min + 1, 1)
    with pytest.raises(fh.FHError):
        batch.select(1, 257)


def test_batch_propose_equals_per_map(batch48):
    # the tiles of all 48 maps through one network, mixed in its batches:
    # every score and every map's top tiles as fh_propose gives them map by map
    import torch
    from paper_1810_09784_amd import fh
    specs, pms, plans, maps, batch = batch48
    net = fh.CNN(max_batch=64)
    rng = np.random.default_rng(4)
    net.set_params(rng.normal(0.0, 0.08, net.n_params).astype(np.float32))
    n_tiles = [((p.n_k + 63) // 64) * ((p.n_x0 + 63) // 64) for p in plans]
    tops = [min(t, 1 + i % 3) for i, t in enumerate(n_tiles)]
    scores, best = fh.fh_batch_propose(net, batch, tops)
    at = 0
    for pl, H, t, k, b in zip(plans, maps, n_tiles, tops, best):
        s1, ids = fh.fh_propose(net, pl, H, k)
        assert torch.equal(scores[at:at + t], s1)
        assert ids == b
        at += t
    assert at == scores.numel()
