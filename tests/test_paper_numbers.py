"""Measurement conventions pinned to the numbers the paper prints (CPU only).

The flop model (Sec. III) and the byte model (Sec. IV transfer volumes) are the
conventions the benchmark reports in; here they must reproduce the paper's own
figures, stored verbatim in ``tests/golden/paper_numbers.json``.
"""
import json
import os

import pytest

from paper_2107_13500_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


def test_flop_model_reproduces_theoretical_gflops(paper):
    fm = paper["flop_model"]
    assert metrics.FLOPS_PER_CELL == fm["flops_per_cell"] == 3 * fm["flops_per_field_stage"]
    assert metrics.FLOPS_COLUMN_TOP == fm["flops_column_top"]
    for clock, printed in fm["theoretical_gflops"].items():
        got = metrics.theoretical_gflops(float(clock), fm["column_height"])
        assert round(got, 2) == printed


def test_table1_percentages_are_consistent(paper):
    t = paper["table_1"]
    th = {k: metrics.theoretical_gflops(float(c)) for k, c in (("u280", 300e6), ("s10", 398e6))}
    for dev in ("u280", "s10"):
        assert round(100 * t[dev] / th[dev]) == t["pct_theoretical"][dev]
    for dev in ("u280", "s10"):
        assert round(100 * t[dev] / t["cpu_24core"]) == t["pct_cpu"][dev]
    # printed as "2400%" for 367.2 / 15.2 = 24.2x
    assert abs(100 * t["v100"] / t["cpu_24core"] - t["pct_cpu"]["v100"]) < 50


def test_table2_overheads(paper):
    for row in paper["table_2"]["rows"]:
        assert round(100 * (row["hbm2"] / row["ddr"] - 1)) == row["overhead_pct"]


def test_ddr_fraction_of_theoretical(paper):
    ddr16 = [r for r in paper["table_2"]["rows"] if r["points"] == "16M"][0]["ddr"]
    assert round(100 * ddr16 / metrics.theoretical_gflops(300e6)) == paper["discussion"]["u280_ddr_pct_theoretical"]


def test_byte_model_reproduces_transfer_volumes(paper):
    for row in paper["transfer_volumes"]["rows"]:
        got = metrics.transfer_bytes_f64(2 ** row["points_log2"])
        # printed to two significant figures (0.8 GB, 3.2 GB, 12.8 GB, 25.8 GB)
        assert abs(got - row["bytes"]) / row["bytes"] < 0.01


def test_algorithmic_bytes_headline_grid():
    # 2048 x 2048 x 64 FP64: 3 halo'd inputs + 3 outputs + 4 coefficient arrays
    b = metrics.algorithmic_bytes(2048, 2048, 64)
    assert b == 8 * (3 * 2050 * 2050 * 64 + 3 * 2048 * 2048 * 64) + 4 * 64 * 8
    assert b == 12_897_492_992
