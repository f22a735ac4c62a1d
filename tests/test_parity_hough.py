"""GPU Hough maps against the oracle, element by element (exact int32).

Runs through the C ABI (fh_plan / fh_hough / fh_batch_*) on the seeded
synthetic peakmaps that both sides consume."""
import math
import sys

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


def _to_dev(pm, dev):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(pm.row_ptr)).to(dev),
            torch.from_numpy(np.ascontiguousarray(pm.bin)).to(dev))


def assert_maps_equal(got, ref, what=""):
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        r, b = bad[0]
        raise AssertionError(f"{what}: {len(bad)} cells differ; first at row {r} col {b}: "
                             f"gpu {got[r, b]} oracle {ref[r, b]}")


def run_gpu(spec_or_desc, pm, dev, tile=None, t=None, n_x0=0, x0_min=0.0, dx0=0.0):
    from paper_1810_09784_amd import fh
    import torch
    s = spec_or_desc
    try:
        plan = fh.Plan(s.n, s.tfft, s.f_min, s.f_max, s.n_fft, s.k, t=t, n_x0=n_x0, x0_min=x0_min, dx0=dx0,
                       tile=tile)
    except fh.FHError as e:  # a tile shape larger than LDS for this map: not applicable
        if e.status == fh.FH_ERANGE and tile is not None:
            return None, None, None
        raise
    rp, bn = _to_dev(pm, dev)
    out = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)  # poison: every cell is written
    fh.fh_hough(plan, rp, bn, out)
    torch.cuda.synchronize()
    return plan, out.cpu().numpy(), fh.fh_device_errors(plan)


def test_tables_match_oracle_bit_for_bit(dev, oracle):
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(5)
    specs = [S.cfg_single_small(), S.cfg_single_large(n_fft=100)] + S.cfg_batched()[:6]
    for _ in range(6):
        specs.append(S.cfg_tiny(rng, n_fft=int(rng.integers(1, 50)), n_f=int(rng.integers(3, 300)),
                                n_k=int(rng.integers(1, 40)), n=float(rng.uniform(1.2, 6.0)),
                                tfft=float(rng.choice([0.5, 1, 2, 4, 8])), f_min=float(rng.integers(200, 2000))))
    for s in specs:
        plan = fh.Plan.from_spec(s)
        d = oracle.Desc.from_spec(s)
        nf, x0m, dx, nx = oracle.grid(d)
        assert (plan.n_f, plan.n_x0) == (nf, nx)
        assert plan.info.x0_min == x0m and plan.info.dx0 == dx
        A, Cr, T = plan.tables()
        Ao, Co, To = oracle.tables(d)
        assert np.array_equal(A.view(np.uint64), Ao.view(np.uint64)), s.name
        assert np.array_equal(Cr.view(np.uint64), Co.view(np.uint64)), s.name
        assert np.array_equal(T.view(np.uint64), To.view(np.uint64)), s.name


@pytest.mark.parametrize("noiseless", [True, False])
def test_single_small_map_exact(dev, oracle, noiseless):
    spec = S.cfg_single_small(noiseless=noiseless)
    pm = S.make_peakmap(spec)
    ref = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin)
    plan, got, errs = run_gpu(spec, pm, dev)
    print(spec.name, plan.tile, file=sys.stderr)
    assert errs == 0
    assert_maps_equal(got, ref, spec.name)
    if noiseless:
        assert got[64].max() == pm.n_peaks == got.max()


TILES = [
    None,
    dict(mode=1, rows=1, cols=64, threads=256, tsplit=1),
    dict(mode=1, rows=3, cols=100, threads=512, tsplit=3),
    dict(mode=1, rows=64, cols=4096, threads=256, tsplit=1),
    dict(mode=1, rows=17, cols=333, threads=256, tsplit=7),
    dict(mode=2, rows=1, cols=37, threads=256, tsplit=1),
    dict(mode=2, rows=2, cols=128, threads=512, tsplit=2),
    dict(mode=2, rows=5, cols=1000, threads=256, tsplit=1),
    dict(mode=1, rows=8, cols=300, threads=1024, tsplit=2),
    dict(mode=2, rows=1, cols=2000, threads=1024, tsplit=4),
]


@pytest.mark.parametrize("seed", range(10))
def test_random_shapes_all_tile_shapes(dev, oracle, seed):
    rng = np.random.default_rng(1000 + seed)
    n = float(rng.choice([1.5, 2.0, 2.5, 3.0, 4.0, 5.0, 7.0]))
    tfft = float(rng.choice([1.0, 2.0, 4.0, 8.0]))
    spec = S.cfg_tiny(rng, n_fft=int(rng.integers(1, 400)), n_f=int(rng.integers(3, 260)),
                      n_k=int(rng.integers(1, 70)), n=n, tfft=tfft, f_min=float(rng.integers(30, 1500)),
                      kscale=float(rng.choice([1e-3, 1e-2, 0.1, 1.0])))
    if seed % 3 == 0:
        pm = S.random_peakmap(rng, spec.n_fft, spec.n_f, float(rng.uniform(0.01, 0.5)))
    else:
        pm = S.make_peakmap(spec)
    ref = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin)
    for tile in TILES:
        plan, got, errs = run_gpu(spec, pm, dev, tile=tile)
        if plan is None:
            continue
        assert errs == 0
        assert_maps_equal(got, ref, f"{spec.name} n={n} tile={plan.tile}")


def test_explicit_times_with_gaps(dev, oracle):
    rng = np.random.default_rng(77)
    spec = S.cfg_tiny(rng, n_fft=500, n_f=150, n_k=40, n=4.0, tfft=2.0, f_min=700.0, kscale=0.3)
    pm = S.make_peakmap(spec)
    t = np.cumsum(rng.uniform(1.0, 9.0, spec.n_fft)) + 3.0  # uneven, with gaps
    ref = oracle.hough(oracle.Desc.from_spec(spec, t=t), pm.row_ptr, pm.bin)
    for tile in TILES[:6]:
        plan, got, errs = run_gpu(spec, pm, dev, tile=tile, t=t)
        if plan is None:
            continue
        assert_maps_equal(got, ref, f"explicit t, tile={plan.tile}")


def test_custom_x0_grid(dev, oracle):
    # a sub-grid (region of interest): explicit x0_min, dx0 and n_x0
    rng = np.random.default_rng(78)
    spec = S.cfg_tiny(rng, n_fft=300, n_f=200, n_k=24, n=3.0, tfft=4.0, f_min=400.0, kscale=0.2)
    pm = S.make_peakmap(spec)
    d0 = oracle.Desc.from_spec(spec)
    nf, x0m, dx, nx = oracle.grid(d0)
    kw = dict(x0_min=x0m + 37.25 * dx, dx0=dx / 3.0, n_x0=nx)
    ref = oracle.hough(oracle.Desc.from_spec(spec, **kw), pm.row_ptr, pm.bin)
    for tile in TILES[:6]:
        plan, got, errs = run_gpu(spec, pm, dev, tile=tile, **kw)
        if plan is None:
            continue
        assert_maps_equal(got, ref, f"custom grid tile={plan.tile}")


def test_bad_bins_skipped_and_counted(dev, oracle):
    rng = np.random.default_rng(79)
    spec = S.cfg_tiny(rng, n_fft=60, n_f=90, n_k=8, n=5.0, tfft=2.0, f_min=500.0, kscale=0.1)
    pm = S.make_peakmap(spec)
    b = pm.bin.copy()
    # FFT 0 gets a negative bin first, the last FFT a too-large bin last (order kept ascending)
    rp = pm.row_ptr.astype(np.int64)
    b_new = np.concatenate([[-5], b[:rp[-1]], [spec.n_f + 3]]).astype(np.int32)
    rp_new = rp + 1
    rp_new[0] = 0
    rp_new[-1] += 1
    ref, bad = oracle.hough(oracle.Desc.from_spec(spec), rp_new.astype(np.int32), b_new, return_bad=True)
    assert bad == 2
    for tile in (None, TILES[1], TILES[5]):
        plan, got, errs = run_gpu(spec, S.Peakmap(rp_new.astype(np.int32), b_new, spec.n_fft, spec.n_f), dev,
                                  tile=tile)
        assert errs == 2, (errs, plan.tile)
        assert_maps_equal(got, ref, "bad bins")


@pytest.mark.parametrize("n_f", [7000, 16000, 17000])
def test_wide_bands_every_rank_build_path(dev, oracle, n_f):
    # windowed maps whose rank structure has 219 words (groups of 4 FFTs in the
    # rank build), 501 words (one FFT per group, past the LDS target) and 532
    # words (above the LDS limit: the per-(FFT, word) search), each with a
    # negative bin first and a too-large bin last, which both paths count
    rng = np.random.default_rng(81 + n_f)
    spec = S.cfg_tiny(rng, n_fft=24, n_f=n_f, n_k=5, n=3.0, tfft=16.0, f_min=2000.0, kscale=0.05)
    pm = S.make_peakmap(spec)
    rp = pm.row_ptr.astype(np.int64)
    b_new = np.concatenate([[-5], pm.bin[:rp[-1]], [spec.n_f + 3]]).astype(np.int32)
    rp_new = rp + 1
    rp_new[0] = 0
    rp_new[-1] += 1
    pm2 = S.Peakmap(rp_new.astype(np.int32), b_new, spec.n_fft, spec.n_f)
    ref, bad = oracle.hough(oracle.Desc.from_spec(spec), pm2.row_ptr, pm2.bin, return_bad=True)
    assert bad == 2
    for tile in (None, dict(mode=2, rows=1, cols=4096, threads=256, tsplit=4),
                 dict(mode=2, rows=2, cols=12000, threads=1024, tsplit=1)):
        plan, got, errs = run_gpu(spec, pm2, dev, tile=tile)
        if plan is None:
            continue
        assert plan.tile["mode"] == 2, plan.tile
        assert errs == 2, (errs, plan.tile)
        assert_maps_equal(got, ref, f"n_f={n_f} tile={plan.tile}")


def test_empty_and_sparse_peakmaps(dev, oracle):
    rng = np.random.default_rng(80)
    spec = S.cfg_tiny(rng, n_fft=50, n_f=40, n_k=5, n=3.0, tfft=1.0, f_min=100.0)
    empty = S.Peakmap(np.zeros(51, dtype=np.int32), np.zeros(0, dtype=np.int32), 50, 40)
    for tile in (None, TILES[2], TILES[5]):
        plan, got, errs = run_gpu(spec, empty, dev, tile=tile)
        assert (got == 0).all()
    one = S.Peakmap(np.r_[np.zeros(26, dtype=np.int32), np.ones(25, dtype=np.int32)], np.array([17], np.int32),
                    50, 40)
    ref = oracle.hough(oracle.Desc.from_spec(spec), one.row_ptr, one.bin)
    for tile in (None, TILES[2], TILES[5]):
        plan, got, errs = run_gpu(spec, one, dev, tile=tile)
        assert_maps_equal(got, ref, "one peak")


def test_deterministic(dev):
    spec = S.cfg_single_small()
    pm = S.make_peakmap(spec)
    _, a, _ = run_gpu(spec, pm, dev)
    _, b, _ = run_gpu(spec, pm, dev)
    assert np.array_equal(a, b)


def test_large_map_sampled_rows(dev, oracle):
    # the 1024 x 84000 map of the 2-day, 200-1200 Hz, n = 3 workload, in the
    # launch configuration the benchmark times; rows sampled for the oracle
    import torch
    from paper_1810_09784_amd import fh
    spec = S.cfg_single_large()
    pm = S.make_peakmap(spec)
    plan = fh.Plan.from_spec(spec)
    assert plan.n_x0 == 84000 and plan.n_k == 1024
    rp, bn = _to_dev(pm, dev)
    out = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    fh.fh_hough(plan, rp, bn, out)
    out2 = torch.empty_like(out)
    fh.fh_hough(plan, rp, bn, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    assert fh.fh_device_errors(plan) == 0
    rows = sorted(set([0, 1, 2, 5, 31, 64, 511, 1023] + list(np.random.default_rng(3).integers(0, 1024, 8))))
    ref = oracle.hough(oracle.Desc.from_spec(spec), pm.row_ptr, pm.bin, rows=rows)
    got = out[rows].cpu().numpy()
    assert_maps_equal(got, ref, "large map rows")
    assert (out >= 0).all().item()


def _batched_inputs(dev, specs):
    import torch
    from paper_1810_09784_amd import fh
    plans, peaks, pms = [], [], []
    for s in specs:
        pm = S.make_peakmap(s)
        pms.append(pm)
        plans.append(fh.Plan.from_spec(s))
        peaks.append(_to_dev(pm, dev))
    return plans, peaks, pms


def test_batched_uneven_maps_exact(dev, oracle):
    # 48 maps: n in {2,2.5,3,4,5,7} x T_FFT in {1,2,4,8} s x 2 seeds, 64 Hz bands,
    # 2 h - 3 days, 64-1024 k rows; one persistent graph launch
    import torch
    from paper_1810_09784_amd import fh
    specs = S.cfg_batched()
    plans, peaks, pms = _batched_inputs(dev, specs)
    maps = [torch.full((p.n_k, p.n_x0), -7, dtype=torch.int32, device=dev) for p in plans]
    ref_maps = [torch.full_like(m, -9) for m in maps]
    batch = fh.Batch(plans, peaks, maps)
    plain = fh.Batch(plans, peaks, ref_maps)
    plain.launch_plain()
    torch.cuda.synchronize()
    for rep in range(3):  # graph replays, with eager work and syncs in between
        for m in maps:
            m.fill_(-7)
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        for q in range(len(maps)):
            assert torch.equal(maps[q], ref_maps[q]), (rep, specs[q].name)
    for q, (s, p) in enumerate(zip(specs, plans)):
        assert fh.fh_device_errors(p) == 0
        rng = np.random.default_rng(q)
        rows = sorted(set([0, s.n_k - 1] + list(rng.integers(0, s.n_k, 3))))
        ref = oracle.hough(oracle.Desc.from_spec(s), pms[q].row_ptr, pms[q].bin, rows=rows)
        assert_maps_equal(maps[q][rows].cpu().numpy(), ref, s.name)
    batch.destroy()
    plain.destroy()


def test_batched_small_maps_full_compare(dev, oracle):
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(90)
    specs = []
    for q in range(12):
        specs.append(S.cfg_tiny(rng, n_fft=int(rng.integers(1, 300)), n_f=int(rng.integers(3, 200)),
                                n_k=int(rng.integers(1, 50)), n=float(rng.choice([2.0, 3.0, 5.0])),
                                tfft=float(rng.choice([1.0, 2.0])), f_min=float(rng.integers(100, 900)),
                                kscale=float(rng.choice([0.01, 0.1, 1.0]))))
    plans, peaks, pms = _batched_inputs(dev, specs)
    # mixed tile shapes in one batch, including windowed and time-split plans
    tiles = [None, TILES[1], TILES[2], TILES[5], TILES[6]]
    plans = [fh.Plan.from_spec(s, tile=tiles[q % len(tiles)]) for q, s in enumerate(specs)]
    maps = [torch.full((p.n_k, p.n_x0), -7, dtype=torch.int32, device=dev) for p in plans]
    fh.fh_hough_batched(plans, peaks, maps)
    torch.cuda.synchronize()
    for q, s in enumerate(specs):
        ref = oracle.hough(oracle.Desc.from_spec(s), pms[q].row_ptr, pms[q].bin)
        assert_maps_equal(maps[q].cpu().numpy(), ref, f"{s.name} tile={plans[q].tile}")


def test_maximum_size_map(dev, oracle):
    # the largest map a plan accepts: n_k n_x0 just below 2^31 cells (8.6 GB of
    # int32), 1023 rows x 2099202 columns of an x0 grid 30000 times finer than
    # the natural one; sampled rows cell by cell, every row's total, and the
    # selection's best cells against the map (properties that hold at any size)
    import torch
    from paper_1810_09784_amd import fh
    rng = np.random.default_rng(81)
    spec = S.cfg_tiny(rng, n_fft=400, n_f=60, n_k=1023, n=3.0, tfft=2.0, f_min=300.0, kscale=0.5)
    pm = S.make_peakmap(spec)
    d0 = oracle.Desc.from_spec(spec)
    nf, x0m, dx, nx = oracle.grid(d0)
    n_x0 = (2**31 - 1) // spec.n_k
    kw = dict(x0_min=x0m, dx0=dx * nx / n_x0, n_x0=n_x0)
    assert spec.n_k * n_x0 < 2**31 <= spec.n_k * (n_x0 + 1)
    plan = fh.Plan(spec.n, spec.tfft, spec.f_min, spec.f_max, spec.n_fft, spec.k, **kw)
    assert (plan.n_k, plan.n_x0) == (spec.n_k, n_x0)
    rp, bn = _to_dev(pm, dev)
    out = torch.full((plan.n_k, plan.n_x0), -7, dtype=torch.int32, device=dev)
    print(f"maximum-size map {plan.n_k} x {plan.n_x0}, tile {plan.tile}", flush=True)
    fh.fh_hough(plan, rp, bn, out)
    torch.cuda.synchronize()
    assert fh.fh_device_errors(plan) == 0
    assert (out.min() >= 0).item()
    d = oracle.Desc.from_spec(spec, **kw)
    rows = sorted(set([0, 1, 7, 8, 63, 64, 511, 1022] + list(rng.integers(0, spec.n_k, 4))))
    ref_rows, _, _ = oracle.rows_checked(d, pm.row_ptr, pm.bin, np.asarray(rows, dtype=np.int32))
    assert_maps_equal(out[rows].cpu().numpy(), ref_rows, "maximum-size map rows")
    _, ref_tot, pairs = oracle.rows_checked(d, pm.row_ptr, pm.bin, np.arange(spec.n_k, dtype=np.int32),
                                            with_map=False)
    assert np.array_equal(out.sum(dim=1, dtype=torch.int64).cpu().numpy(), ref_tot)
    assert int(pairs.sum()) > 0
    # selection: each square's best cell is the square's maximum, first in row-major order
    sq_k, sq_x0 = 5, 5
    cands, n = fh.fh_select(plan, out, sq_k, sq_x0, 3)
    assert n == len(cands) > 0
    for c in cands:
        a, b = divmod(c["square"], sq_x0)
        r0, r1 = a * plan.n_k // sq_k, (a + 1) * plan.n_k // sq_k
        c0, c1 = b * plan.n_x0 // sq_x0, (b + 1) * plan.n_x0 // sq_x0
        assert r0 <= c["row"] < r1 and c0 <= c["col"] < c1
        assert int(out[c["row"], c["col"]]) == c["count"]
        if not c["second"]:
            region = out[r0:r1, c0:c1]
            assert int(region.max()) == c["count"]
            first = torch.nonzero(region == c["count"])[0]
            assert (c["row"], c["col"]) == (int(first[0]) + r0, int(first[1]) + c0)
    del out
    torch.cuda.empty_cache()
