"""Host logic of bench.py's roofline: each kernel is judged against the peak of its own
arithmetic (f32 MFMA, or the dense bf16 peak divided by the bf16 products per algorithmic
product of a split), MFMA-bound above that arithmetic's ridge and HBM-bound below it, and the
reported entry is the (kernel, level) with the most time.  Synthetic per-kernel records."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def rec(kind, level, launches, ms_total, bytes_per_launch, flops_per_launch):
    return dict(kind=kind, level=level, launches=launches, ms_total=ms_total,
                bytes_per_launch=bytes_per_launch, flops_per_launch=flops_per_launch)


def test_matrix_peaks(bench):
    assert bench.matrix_peak("smooth_in", 0, 0)[0] == bench.FP32_PEAK_TFS
    assert bench.matrix_peak("smooth_in", 0, 1)[0] == bench.FP32_PEAK_TFS
    assert bench.matrix_peak("smooth_in", 0, 2)[0] == pytest.approx(bench.BF16_PEAK_TFS / 3)
    assert bench.matrix_peak("smooth_up", 0, 1)[0] == pytest.approx(bench.BF16_PEAK_TFS / 6)
    assert bench.matrix_peak("restrict", 0, 2)[0] == bench.FP32_PEAK_TFS
    assert bench.matrix_peak("prolong", 3, -1)[0] == bench.BF16_PEAK_TFS


def test_bound_follows_the_kernels_own_ridge(bench):
    # 37 flop/B: above the f32 ridge (19.7), below the two-way split's (104)
    stats = [rec("smooth_in", 0, 10, 10.0, 1e9, 37e9), rec("prolong", 0, 10, 5.0, 1e9, 8e9)]
    roof, share, total, _ = bench.roofline_of(stats, split=1)
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    assert roof["achieved"] == pytest.approx(37.0)          # 37e9 flop per 1 ms
    assert roof["frac"] == pytest.approx(37.0 / bench.FP32_PEAK_TFS, abs=1e-4)
    roof, _, _, _ = bench.roofline_of(stats, split=2)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    assert roof["achieved"] == pytest.approx(1000.0)        # 1e9 B per 1 ms
    assert roof["frac"] == pytest.approx(1000.0 / bench.HBM_PEAK_GBS)
    assert total == pytest.approx(15.0)
    assert share == {"smooth_in": pytest.approx(2 / 3, abs=1e-4), "prolong": pytest.approx(1 / 3, abs=1e-4)}


def test_reported_entry_has_the_most_time(bench):
    stats = [rec("smooth_in", 0, 100, 10.0, 8e9, 1e9), rec("smooth_up", 0, 100, 12.0, 12e9, 3e11),
             rec("smooth_up", 1, 400, 11.0, 3e9, 7e10)]
    roof, _, _, level0 = bench.roofline_of(stats, split=2)
    assert roof["kernel"].startswith("smooth_up (level 0")
    assert roof["bound"] == "hbm"                            # 25 flop/B < 52 (three-way split)
    assert set(level0) == {"smooth_in", "smooth_up"}
