"""The fused GEMV's launch planner (host logic, no GPU): every block of the
range is covered exactly by the launch, and the measured rule holds (8 lanes
per block row for square and tall matrices, wider groups for few block rows
(tiles at least 90 % full),
narrower ones for few block columns; 2048-ish workgroups; few slabs on
large matrices)."""
import math

import pytest

from paper_1902_08018_amd import wh

SHAPES = [(65536, 65536, 0, 65536), (65536, 65536, 0, 8192), (16384, 16384, 0, 16384), (378, 256000, 0, 378),
          (256000, 378, 0, 256000), (10000, 10000, 0, 10000), (2116, 256000, 401, 779), (1, 1, 0, 1),
          (5, 7, 1, 4), (61, 4100, 3, 59), (4096, 12, 0, 4096), (33, 2, 0, 33)]


@pytest.mark.parametrize("rows,cols,rb,re", SHAPES)
def test_plan_covers_the_range(rows, cols, rb, re):
    p = wh.wh_gemv_plan_info(rows, cols, rb, re)
    nbc = (cols + 3) // 4
    assert p["bi_begin"] == rb // 4 and p["bi_end"] == (re + 3) // 4 and p["skip"] == rb % 4
    lanes = p["lanes"]
    assert lanes in (4, 8, 16, 32, 64, 128, 256, 512) and p["rows_per_group"] in (1, 2, 4)
    # rows: tiles of (workgroup lanes / lanes) * rows_per_group block rows
    assert p["wg_lanes"] in (768, 1024)
    tile_rows = (p["wg_lanes"] // lanes) * p["rows_per_group"]
    assert p["ntiles"] * tile_rows >= p["bi_end"] - p["bi_begin"] > (p["ntiles"] - 1) * tile_rows
    # columns: slabs of whole lane groups, the last one non-empty
    assert p["slab_bc"] % lanes == 0
    assert p["nslab"] * p["slab_bc"] >= nbc > (p["nslab"] - 1) * p["slab_bc"]


def test_measured_rule():
    big = wh.wh_gemv_plan_info(65536, 65536)
    assert big["lanes"] == 8 and big["rows_per_group"] == 1 and big["nslab"] <= 64
    slit = wh.wh_gemv_plan_info(378, 256000)
    assert slit["lanes"] == 32 and slit["ntiles"] == 3          # 95 block rows in 32-row tiles
    tall = wh.wh_gemv_plan_info(256000, 378)
    assert tall["lanes"] == 8 and tall["nslab"] <= 4            # 95 block columns, ~2000 workgroups
    narrow = wh.wh_gemv_plan_info(4096, 12)
    assert narrow["lanes"] == 4                                  # 3 block columns
    for shape in [(16384, 16384), (10000, 10000), (32768, 16384)]:
        p = wh.wh_gemv_plan_info(*shape)
        assert 1000 <= p["ntiles"] * p["nslab"] <= 5000


def test_plan_errors():
    with pytest.raises(wh.WhError):
        wh.wh_gemv_plan_info(8, 8, 5, 4)
    with pytest.raises(wh.WhError):
        wh.wh_gemv_plan_info(8, 8, 0, 9)
