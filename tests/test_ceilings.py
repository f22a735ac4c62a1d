"""The measured-ceilings microbenchmark: the stored MI355X measurement is
complete and below the data-sheet peaks; on a GPU it runs again and agrees
with itself to within clock and thermal drift."""
import pytest

from paper_1810_09784_amd import ceilings

TESTS = {
    # test -> (field, data-sheet bound for MI355X)
    "fp64_fma": ("tflops", 78.6),
    "fp64_fma_plus_cvt_i32": ("g_pairs_per_s", 78.6e3 / 2),
    "lds_atomic_add_consecutive": ("g_lane_ops_per_s", 64 * 256 * 2.4),
    "lds_atomic_add_random": ("g_lane_ops_per_s", 64 * 256 * 2.4),
    "lds_atomic_add_one_bank": ("g_lane_ops_per_s", 64 * 256 * 2.4),
    "hbm_read_1GiB": ("gb_per_s", 8000.0),
    "hbm_copy_1GiB": ("gb_per_s", 8000.0),
    "hbm_store_1GiB": ("gb_per_s", 8000.0),
    "mfma_bf16_16x16x32": ("tflops", 2500.0),
    # 32-bit integer adds issue faster than one wave instruction per CU cycle
    # (measured about 1.7 at the nominal clock); two per cycle bounds them
    "valu_issue_i32": ("g_wave_instr_per_s", 2 * 256 * 2.4),
}


def _check(res):
    assert res["device"]["arch"].startswith("gfx950")
    for name, (field, bound) in TESTS.items():
        v = res["tests"][name][field]
        assert 0 < v <= bound, (name, v, bound)
    t = res["tests"]
    # one bank serialises the 64 lanes: far below the scattered patterns
    assert t["lds_atomic_add_one_bank"]["g_lane_ops_per_s"] < 0.25 * t["lds_atomic_add_random"]["g_lane_ops_per_s"]


def test_stored_measurement_complete_and_below_datasheet():
    res = ceilings.load()
    assert res is not None, "ceilings_gfx950.json missing"
    _check(res)


@pytest.mark.gpu
def test_ceilings_run_on_the_gpu():
    import os
    from paper_1810_09784_amd import build
    if not os.path.exists(build.CEILINGS):
        pytest.skip("microbenchmark not built")
    res = ceilings.run()
    _check(res)
    old = ceilings.load()
    for name in ("hbm_read_1GiB", "lds_atomic_add_random", "mfma_bf16_16x16x32"):
        f = TESTS[name][0]
        assert 0.5 < res["tests"][name][f] / old["tests"][name][f] < 2.0, name
