"""fh_hough_select (the transform with the selection's row pass fused into the
tile kernel's epilogue) against the oracle: its map against the oracle's Hough
map, its candidates against the oracle selection of that map, over tile
shapes that take every epilogue path (whole rows per wave, runs of chunks per
wave, split tiles summarised by the pass after the tile kernel) and both
pair-finding modes."""
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


def _compare(got, ref):
    assert len(got) == len(ref), (len(got), len(ref))
    for g, r in zip(got, ref):
        for key in ("row", "col", "count", "square", "second"):
            assert g[key] == r[key], (key, g, r)
        for key in ("cr", "mu", "sigma", "x0", "k", "f0", "fdot0"):
            assert g[key] == r[key] or (np.isnan(g[key]) and np.isnan(r[key])), (key, g[key], r[key])


def _fused(plan, pm, dev, sq, min_dk=3, thr=-1e300, cols=(0, 0)):
    import torch
    from paper_1810_09784_amd import fh
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    H = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    fh.fh_hough_select(plan, rp, bn, H, sq[0], sq[1], min_dk, thr, col_lo=cols[0], col_hi=cols[1])
    got, n = fh.fh_select_results(plan)
    return H.cpu().numpy(), got, n


# tile shapes: (rows, cols, threads, mode, tsplit).  Small maps split nearly
# every tile over FFT ranges when tsplit > 1 (the unit target is the total
# cost over 4x the resident work-groups).
TILES = [
    None,                                                                   # the plan's own choice
    dict(rows=1, cols=100, threads=1024, mode=1, tsplit=1),                 # runs of chunks per wave, no split
    dict(rows=1, cols=100, threads=1024, mode=1, tsplit=8),                 # split tiles, read back after
    dict(rows=8, cols=64, threads=256, mode=2, tsplit=1),                   # whole rows per wave, windowed
    dict(rows=12, cols=80, threads=512, mode=2, tsplit=16),                 # whole rows per wave, split
    dict(rows=3, cols=323, threads=256, mode=2, tsplit=4),                  # one column tile, few rows
]


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("sq,min_dk,thr,cols", [((5, 5), 3, -1e300, (0, 0)), ((8, 3), 3, 2.0, (0, 0)),
                                                ((4, 37), 5, 0.0, (30, 300)), ((1, 256), 0, -1e300, (0, 0))])
def test_fused_small_map(dev, oracle, tile, sq, min_dk, thr, cols):
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    spec = S.cfg_single_small()
    pm = S.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec, tile=tile)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    got_map, got, n = _fused(plan, pm, dev, sq, min_dk, thr, cols)
    assert np.array_equal(got_map, ref_map)
    nf, x0m, dx, nx = oracle.grid(d)
    ref = OS.select(ref_map, spec.k, x0m, dx, spec.n, sq[0], sq[1], min_dk, thr, cols[0], cols[1])
    assert n == len(ref)
    _compare(got, ref)


@pytest.mark.parametrize("seed", range(6))
def test_fused_random_maps_with_ties(dev, oracle, seed):
    # unstructured peaks, small counts (many ties), one-column segments and
    # random tile shapes
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    rng = np.random.default_rng(900 + seed)
    spec = S.cfg_tiny(rng, n_fft=int(rng.integers(20, 300)), n_f=int(rng.integers(20, 160)),
                      n_k=int(rng.integers(8, 90)), n=float(rng.choice([2.0, 3.0, 5.0])), tfft=2.0,
                      f_min=float(rng.integers(100, 800)), kscale=0.05)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.05)
    probe = fh.Plan.from_spec(spec)
    nx = probe.n_x0
    tile = dict(rows=int(rng.integers(1, 20)), cols=int(rng.integers(1, nx + 1)),
                threads=int(rng.choice([256, 512, 1024])), mode=int(rng.choice([1, 2])),
                tsplit=int(rng.choice([1, 3, 16])))
    plan = fh.Plan.from_spec(spec, tile=tile)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    sk = int(rng.integers(1, min(8, spec.n_k) + 1))
    sx = nx if seed == 0 and nx <= 256 else int(rng.integers(1, min(40, nx) + 1))
    got_map, got, n = _fused(plan, pm, dev, (sk, sx))
    assert np.array_equal(got_map, ref_map), tile
    nf, x0m, dx, _ = oracle.grid(d)
    _compare(got, OS.select(ref_map, spec.k, x0m, dx, spec.n, sk, sx, 3))


def test_fused_large_map(dev, oracle):
    # the full 1024 x 84000 map (windowed mode, split tiles) and 5 x 5 squares
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    spec = S.cfg_single_large()
    pm = S.make_peakmap(spec)
    from paper_1810_09784_amd import tune
    plan = fh.Plan.from_spec(spec, tile=tune.lookup(spec, pm.n_peaks))  # the benchmark's launch configuration
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    got_map, got, n = _fused(plan, pm, dev, (5, 5))
    bad = np.argwhere(got_map != ref_map)
    assert len(bad) == 0, f"{len(bad)} cells differ, first {bad[:3]}"
    nf, x0m, dx, nx = oracle.grid(d)
    _compare(got, OS.select(ref_map, spec.k, x0m, dx, spec.n, 5, 5, 3))
    # 7 x 256 squares on the same map: segments far narrower than a tile
    got_map, got, n = _fused(plan, pm, dev, (7, 256), 2, 3.0)
    assert np.array_equal(got_map, ref_map)
    ref = OS.select(ref_map, spec.k, x0m, dx, spec.n, 7, 256, 2, 3.0)
    assert n == len(ref)
    _compare(got, ref)


@pytest.mark.parametrize("n_streams", [1, 2])
def test_fused_pipelined_two_plans(dev, oracle, n_streams):
    # two plans of one description alternate over four peakmaps, on one stream
    # or one stream each; each call's results are fetched after the next call
    # was enqueued
    import torch
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    specs = [S.cfg_single_small(seed=s) for s in (11, 12, 13, 14)]
    plans = [fh.Plan.from_spec(specs[0]), fh.Plan.from_spec(specs[0])]
    maps = [torch.empty((plans[0].n_k, plans[0].n_x0), dtype=torch.int32, device=dev) for _ in range(2)]
    inputs = []
    for sp in specs:
        pm = S.make_peakmap(sp)
        inputs.append((pm, torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev)))
    d = oracle.Desc.from_spec(specs[0])
    nf, x0m, dx, nx = oracle.grid(d)
    streams = [torch.cuda.current_stream()]
    if n_streams == 2:
        streams.append(torch.cuda.Stream())
        streams[1].wait_stream(streams[0])  # the inputs and maps were written on the first
    results = []
    for i, (pm, rp, bn) in enumerate(inputs):
        fh.fh_hough_select(plans[i % 2], rp, bn, maps[i % 2], 6, 4, 3, stream=streams[i % n_streams])
        if i >= 1:
            results.append(fh.fh_select_results(plans[(i - 1) % 2]))
    results.append(fh.fh_select_results(plans[(len(inputs) - 1) % 2]))
    streams[0].wait_stream(streams[-1])
    for (pm, _, _), (got, n) in zip(inputs, results):
        ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
        _compare(got, OS.select(ref_map, specs[0].k, x0m, dx, specs[0].n, 6, 4, 3))
    # nothing pending now
    with pytest.raises(fh.FHError):
        fh.fh_select_results(plans[0])


def test_fused_rejects_bad_options(dev):
    import torch
    from paper_1810_09784_amd import fh
    spec = S.cfg_single_small()
    pm = S.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    H = torch.zeros((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
    for kw in (dict(sq_k=0, sq_x0=1), dict(sq_k=1, sq_x0=0), dict(sq_k=plan.n_k + 1, sq_x0=1),
               dict(sq_k=1, sq_x0=1, col_lo=10, col_hi=5), dict(sq_k=1, sq_x0=300)):
        with pytest.raises(fh.FHError):
            fh.fh_hough_select(plan, rp, bn, H, **kw)
    with pytest.raises(fh.FHError):
        fh.fh_select_results(plan)


def test_fused_empty_peakmap_and_bad_bins(dev, oracle):
    # no peaks at all: an all-zero map, sigma = 0 everywhere, no candidate;
    # then bins outside [0, n_f): skipped in the map and counted as errors
    import torch
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    rng = np.random.default_rng(77)
    spec = S.cfg_tiny(rng, n_fft=64, n_f=40, n_k=20, n=3.0, kscale=0.05)
    plan = fh.Plan.from_spec(spec, tile=dict(rows=4, cols=16, threads=256, mode=2, tsplit=4))
    empty = S.Peakmap(row_ptr=np.zeros(spec.n_fft + 1, dtype=np.int32), bin=np.zeros(0, dtype=np.int32),
                      n_fft=spec.n_fft, n_f=spec.n_f)
    got_map, got, n = _fused(plan, empty, dev, (2, 3))
    assert not got_map.any() and n == 0 and got == []
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.1)
    bins = pm.bin.copy()
    bins[::7] = spec.n_f + 3  # out of range (ascending order is not kept for these FFTs)
    bad = S.Peakmap(row_ptr=pm.row_ptr, bin=bins, n_fft=pm.n_fft, n_f=pm.n_f)
    keep = bins < spec.n_f
    counts = np.diff(pm.row_ptr)
    fft_of = np.repeat(np.arange(spec.n_fft), counts)
    rp_ok = np.zeros(spec.n_fft + 1, dtype=np.int32)
    np.cumsum(np.bincount(fft_of[keep], minlength=spec.n_fft), out=rp_ok[1:])
    ref_map = oracle.hough(oracle.Desc.from_spec(spec), rp_ok, bins[keep])
    plan_w = fh.Plan.from_spec(spec, tile=dict(rows=4, cols=16, threads=256, mode=1, tsplit=4))
    got_map, got, n = _fused(plan_w, bad, dev, (2, 3))  # whole-FFT mode: order within an FFT is irrelevant
    assert np.array_equal(got_map, ref_map)
    # bad peaks: out of the band, or not above the previous bin of their FFT (the
    # peak after each planted bin counts too), each once
    first = np.zeros(bins.size, dtype=bool)
    first[pm.row_ptr[:-1][counts > 0]] = True
    prev = np.concatenate([[0], bins[:-1]])
    n_bad = int(np.sum(~keep | (~first & (bins <= prev))))
    assert n_bad > int((~keep).sum())
    assert fh.fh_device_errors(plan_w) == n_bad
    nf, x0m, dx, nx = oracle.grid(oracle.Desc.from_spec(spec))
    _compare(got, OS.select(ref_map, spec.k, x0m, dx, spec.n, 2, 3, 3))


@pytest.mark.parametrize("cols", [1, 7, 300])
def test_fused_one_column_segments(dev, oracle, cols):
    # as many squares along x0 as analysed columns (every segment one column
    # wide, boundaries inside every step), on narrow and wide tiles
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    rng = np.random.default_rng(5150 + cols)
    spec = S.cfg_tiny(rng, n_fft=150, n_f=60, n_k=24, n=2.0, kscale=0.05)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.08)
    plan = fh.Plan.from_spec(spec, tile=dict(rows=2, cols=cols, threads=512, mode=2, tsplit=2))
    nx = plan.n_x0
    lo, hi = 1, min(nx, 1 + 256)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    got_map, got, n = _fused(plan, pm, dev, (3, hi - lo), 2, -1e300, (lo, hi))
    assert np.array_equal(got_map, ref_map)
    nf, x0m, dx, _ = oracle.grid(d)
    ref = OS.select(ref_map, spec.k, x0m, dx, spec.n, 3, hi - lo, 2, -1e300, lo, hi)
    assert n == len(ref)
    _compare(got, ref)


def test_fused_pending_results_and_plain_select(dev, oracle):
    # a plain fh_select on the same plan while fused results are pending leaves
    # them fetchable; a second fused call drops unfetched results of the first
    import torch
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    specs = [S.cfg_single_small(seed=s) for s in (21, 22)]
    plan = fh.Plan.from_spec(specs[0])
    d = oracle.Desc.from_spec(specs[0])
    nf, x0m, dx, nx = oracle.grid(d)
    pms = [S.make_peakmap(sp) for sp in specs]
    dev_pk = [(torch.from_numpy(p.row_ptr).to(dev), torch.from_numpy(p.bin).to(dev)) for p in pms]
    refs = [oracle.hough(d, p.row_ptr, p.bin) for p in pms]
    H0 = torch.empty((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
    H1 = torch.from_numpy(refs[1]).to(dev)
    fh.fh_hough_select(plan, *dev_pk[0], H0, 4, 4, 3)
    plain, _ = fh.fh_select(plan, H1, 3, 5, 2)
    _compare(plain, OS.select(refs[1], specs[0].k, x0m, dx, specs[0].n, 3, 5, 2))
    got, _ = fh.fh_select_results(plan)
    _compare(got, OS.select(refs[0], specs[0].k, x0m, dx, specs[0].n, 4, 4, 3))
    fh.fh_hough_select(plan, *dev_pk[0], H0, 4, 4, 3)
    fh.fh_hough_select(plan, *dev_pk[1], H0, 2, 6, 3)  # the first call's results are dropped
    got, _ = fh.fh_select_results(plan)
    _compare(got, OS.select(refs[1], specs[0].k, x0m, dx, specs[0].n, 2, 6, 3))
    with pytest.raises(fh.FHError):
        fh.fh_select_results(plan)
