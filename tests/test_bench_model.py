"""The benchmark's algorithmic byte model (host only): the direct-probe
counts it charges per kernel follow the method's own counts."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def counts(pos=1000, cand=400, popcount=0):
    return {"positions": pos, "edge_positions": pos - 1, "candidates": cand, "junctions": 100,
            "edges": 99, "bloom_popcount": popcount}


BIG = 1 << 33  # beyond the last-level cache: probes are charged


def test_blocked_query_one_block_per_position():
    c = counts()
    out, probes, where = bench.algorithmic_bytes(c, 1000, 25, 1, 5, True, BIG, BIG, 0)
    assert probes["query"] == 1000 and where["filter_in_hbm"]
    assert out["query"] == pytest.approx(1000 / 4 + 1000 / 8 + bench.GRANULE * 1000)


@pytest.mark.parametrize("r,h,per", [(0.0, 5, 6.0), (0.5, 2, 9.0), (0.5, 3, 10.5)])
def test_standard_query_stops_at_the_first_clear_bit(r, h, per):
    # a membership test reads bit t only when bits 0..t-1 were set: the
    # expected words per test are 1 + r + ... + r^(h-1), six tests per position
    c = counts(popcount=int(r * BIG * 8))
    _, probes, _ = bench.algorithmic_bytes(c, 1000, 25, 1, h, False, BIG, BIG, 0)
    assert probes["query"] == pytest.approx(1000 * per)


def test_saturated_standard_filter_tests_every_bit():
    c = counts(popcount=BIG * 8)
    _, probes, _ = bench.algorithmic_bytes(c, 1000, 25, 1, 4, False, BIG, BIG, 0)
    assert probes["query"] == pytest.approx(1000 * 6 * 4, rel=1e-6)


def test_structures_in_the_last_level_cache_cost_no_probe_bytes():
    c = counts()
    small = bench.MALL_BYTES // 2
    out, _, where = bench.algorithmic_bytes(c, 1000, 25, 1, 5, True, small, small, 0)
    assert not where["filter_in_hbm"] and not where["table_in_hbm"]
    assert out["query"] == pytest.approx(1000 / 4 + 1000 / 8)
    assert out["record"] == pytest.approx(1000 / 4 + 1000 / 8)
