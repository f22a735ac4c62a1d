"""fh_select (GPU pass + host finish) against the oracle selection run on the
oracle's own Hough map."""
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


def _gpu_map(spec, pm, dev, plan):
    import torch
    from paper_1810_09784_amd import fh
    rp = torch.from_numpy(pm.row_ptr).to(dev)
    bn = torch.from_numpy(pm.bin).to(dev)
    return fh.fh_hough(plan, rp, bn)


def _compare(got, ref):
    assert len(got) == len(ref), (len(got), len(ref))
    for g, r in zip(got, ref):
        for key in ("row", "col", "count", "square", "second"):
            assert g[key] == r[key], (key, g, r)
        for key in ("cr", "mu", "sigma", "x0", "k", "f0", "fdot0"):
            assert g[key] == r[key] or (np.isnan(g[key]) and np.isnan(r[key])), (key, g[key], r[key])


@pytest.mark.parametrize("sq,min_dk,thr,cols", [((5, 5), 3, -1e300, (0, 0)), ((8, 3), 3, 2.0, (0, 0)),
                                                ((1, 1), 0, -1e300, (0, 0)), ((4, 6), 5, 0.0, (30, 300))])
def test_select_small_map(dev, oracle, sq, min_dk, thr, cols):
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    spec = S.cfg_single_small()
    pm = S.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    H = _gpu_map(spec, pm, dev, plan)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    assert np.array_equal(H.cpu().numpy(), ref_map)
    got, n = fh.fh_select(plan, H, sq[0], sq[1], min_dk, thr, col_lo=cols[0], col_hi=cols[1])
    nf, x0m, dx, nx = oracle.grid(d)
    ref = OS.select(ref_map, spec.k, x0m, dx, spec.n, sq[0], sq[1], min_dk, thr, cols[0], cols[1])
    assert n == len(ref)
    _compare(got, ref)
    if sq == (5, 5) and thr < 0:
        best = max(got, key=lambda c: c["cr"])  # the injection: k row 64, f0 = 580 Hz
        assert best["row"] == 64 and abs(best["f0"] - 580.0) < 0.5


@pytest.mark.parametrize("seed", range(4))
def test_select_random_maps_with_ties(dev, oracle, seed):
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    rng = np.random.default_rng(300 + seed)
    spec = S.cfg_tiny(rng, n_fft=int(rng.integers(20, 200)), n_f=int(rng.integers(20, 120)),
                      n_k=int(rng.integers(8, 60)), n=float(rng.choice([2.0, 3.0, 5.0])), tfft=2.0,
                      f_min=float(rng.integers(100, 800)), kscale=0.05)
    pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, 0.05)  # small counts: many ties
    plan = fh.Plan.from_spec(spec)
    H = _gpu_map(spec, pm, dev, plan)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    assert np.array_equal(H.cpu().numpy(), ref_map)
    sk = int(rng.integers(1, min(8, spec.n_k) + 1))
    sx = int(rng.integers(1, min(8, plan.n_x0) + 1))
    got, n = fh.fh_select(plan, H, sk, sx, 3)
    nf, x0m, dx, nx = oracle.grid(d)
    _compare(got, OS.select(ref_map, spec.k, x0m, dx, spec.n, sk, sx, 3))


@pytest.mark.parametrize("n_x0,n_k,sq,cols,hi", [
    (1001, 300, (300, 7), (3, 998), 3),      # one row per square, unaligned column range, many ties
    (4099, 517, (1, 256), (1, 0), 100000),   # 517 rows in one square (strided row loop), 256 segments
    (30001, 64, (5, 5), (0, 0), 50),         # long segments: the 4-deep 16-byte load loop and its tails
    (37, 11, (11, 37), (0, 0), 2),           # one-column segments
    (6, 3, (2, 2), (1, 6), 0),               # all-zero map: sigma = 0, no candidate
])
def test_select_random_integer_maps(dev, n_x0, n_k, sq, cols, hi):
    # maps that fh_hough did not write: any counts, odd widths and column ranges
    import torch
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    k = np.linspace(0.0, 1e-12, n_k)
    plan = fh.Plan(3.0, 2.0, 100.0, 110.0, 4, k, x0_min=1e-4, dx0=1e-7, n_x0=n_x0)
    g = torch.Generator(device=dev)
    g.manual_seed(n_x0 * 7 + n_k)
    H = torch.randint(0, hi + 1, (n_k, n_x0), generator=g, device=dev, dtype=torch.int32)
    got, n = fh.fh_select(plan, H, sq[0], sq[1], 3, col_lo=cols[0], col_hi=cols[1])
    ref = OS.select(H.cpu().numpy(), k, plan.info.x0_min, plan.info.dx0, 3.0, sq[0], sq[1], 3,
                    col_lo=cols[0], col_hi=cols[1])
    assert n == len(ref)
    _compare(got, ref)
    # a second call with fewer squares reuses the scratch
    got2, _ = fh.fh_select(plan, H, 1, 1, 3, col_lo=cols[0], col_hi=cols[1])
    _compare(got2, OS.select(H.cpu().numpy(), k, plan.info.x0_min, plan.info.dx0, 3.0, 1, 1, 3,
                             col_lo=cols[0], col_hi=cols[1]))


def test_large_map_full_parity_and_select(dev, oracle):
    # the whole 1024 x 84000 map against the oracle's, then 5 x 5 squares
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    spec = S.cfg_single_large()
    pm = S.make_peakmap(spec)
    from paper_1810_09784_amd import tune
    plan = fh.Plan.from_spec(spec, tile=tune.lookup(spec, pm.n_peaks))  # the benchmark's launch configuration
    H = _gpu_map(spec, pm, dev, plan)
    d = oracle.Desc.from_spec(spec)
    ref_map = oracle.hough(d, pm.row_ptr, pm.bin)
    got_map = H.cpu().numpy()
    bad = np.argwhere(got_map != ref_map)
    assert len(bad) == 0, f"{len(bad)} cells differ, first {bad[:3]}"
    got, n = fh.fh_select(plan, H, 5, 5, 3)
    nf, x0m, dx, nx = oracle.grid(d)
    _compare(got, OS.select(ref_map, spec.k, x0m, dx, spec.n, 5, 5, 3))


def test_select_rejects_bad_options(dev):
    from paper_1810_09784_amd import fh
    spec = S.cfg_single_small()
    plan = fh.Plan.from_spec(spec)
    import torch
    H = torch.zeros((plan.n_k, plan.n_x0), dtype=torch.int32, device=dev)
    for kw in (dict(sq_k=0, sq_x0=1), dict(sq_k=1, sq_x0=0), dict(sq_k=plan.n_k + 1, sq_x0=1),
               dict(sq_k=1, sq_x0=1, col_lo=10, col_hi=5), dict(sq_k=1, sq_x0=300)):
        with pytest.raises(fh.FHError):
            fh.fh_select(plan, H, **kw)


def _oracle_tile(OS, H, k, x0m, dx, n, t, sq, col_lo=0, col_hi=0):
    """The oracle's selection applied to tile t's rectangle as a map of its own."""
    n_k, n_x0 = H.shape
    tb = (n_x0 + 63) // 64
    a, b = divmod(t, tb)
    r0, r1 = 64 * a, min(64 * a + 64, n_k)
    c0 = max(64 * b, col_lo)
    c1 = min(64 * b + 64, n_x0, col_hi if col_hi > 0 else n_x0)
    if c0 >= c1:
        return []
    sub = np.ascontiguousarray(H[r0:r1])
    out = OS.select(sub, np.asarray(k)[r0:r1], x0m, dx, n, sq[0], sq[1], sq[2], col_lo=c0, col_hi=c1)
    for c in out:
        c["row"] += r0
    return out


def test_select_tiles_against_oracle(dev, oracle):
    import torch
    from paper_1810_09784_amd import fh
    from oracle import select as OS
    spec = S.cfg_single_small()
    pm = S.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    H = fh.fh_hough(plan, torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev))
    ref_map = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin)
    assert np.array_equal(H.cpu().numpy(), ref_map)
    _, x0m, dx, _ = oracle.grid(oracle.Desc.from_spec(spec))
    tiles = [0, 5, 7, 11, 3]  # tile 5 and 11: the last 3 columns of the 323
    keys = ("row", "col", "count", "square", "second", "cr", "mu", "sigma", "x0", "k", "f0", "fdot0")
    for sq, cols in (((2, 1, 3), (0, 0)), ((2, 2, 3), (0, 0)), ((1, 1, 0), (10, 300))):
        got, counts, n = fh.fh_select_tiles(plan, H, tiles, *sq, col_lo=cols[0], col_hi=cols[1])
        ref = []
        for t in tiles:
            r = _oracle_tile(OS, ref_map, spec.k, x0m, dx, spec.n, t, sq, *cols)
            ref += r
            assert counts[tiles.index(t)] == len(r)
        assert n == len(ref) == len(got)
        for g, r in zip(got, ref):
            assert tuple(g[x] for x in keys) == tuple(r[x] for x in keys), (sq, g, r)
    # tile 5 lies outside columns [10, 300): no candidate from it
    _, counts, _ = fh.fh_select_tiles(plan, H, [5], 1, 1, 0, col_lo=10, col_hi=300)
    assert counts[0] == 0
    with pytest.raises(fh.FHError):
        fh.fh_select_tiles(plan, H, [12], 2, 2)  # 2 x 6 tiles: index 12 is outside
    with pytest.raises(fh.FHError):
        fh.fh_select_tiles(plan, H, [0], 65, 1)  # more squares than the tile has rows


def test_batch_select_tiles_equals_per_map(dev):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(23)
    specs = [S.cfg_tiny(rng, n_fft=400, n_f=80 + 40 * i, n_k=70 + 30 * i, n=3.0 + i, f_min=200.0 + 100 * i)
             for i in range(3)]
    plans, peaks, maps = [], [], []
    for s in specs:
        pm = S.make_peakmap(s)
        plans.append(fh.Plan.from_spec(s))
        peaks.append((torch.from_numpy(pm.row_ptr).to(dev), torch.from_numpy(pm.bin).to(dev)))
        maps.append(torch.empty((plans[-1].n_k, plans[-1].n_x0), dtype=torch.int32, device=dev))
    b = fh.Batch(plans, peaks, maps)
    b.launch()
    torch.cuda.synchronize()
    tb = [(p.n_x0 + 63) // 64 for p in plans]
    req = [(0, 1), (2, 2 * tb[2] - 1), (1, 0), (0, 1), (1, tb[1])]
    got, counts, n = b.select_tiles(req, 2, 1, 3, cr_thr=1.5)
    at = 0
    for q, (mi, t) in enumerate(req):
        ref, rc, rn = fh.fh_select_tiles(plans[mi], maps[mi], [t], 2, 1, 3, cr_thr=1.5, as_dicts=False)
        assert counts[q] == rn == rc[0]
        assert np.array_equal(got[at:at + rn], ref)
        at += rn
    assert at == n
    b.destroy()
