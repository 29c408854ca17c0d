"""Runtime knobs and the autotuner: outputs are bit-identical under every
configuration (workgroups per CU, first-pass tile order, table load factor,
including loads that force the exact tables to regrow), and the tuner's
cache is written and reused."""
import os
import sys

import numpy as np
import pytest

import synth
from helpers import to_genomes

pytestmark = pytest.mark.gpu

BLOCKED = 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05856_amd as tp
    tp.lib()


def outputs(plan, d_in):
    plan.run(d_in)
    r = plan.download()
    return (r.junction_offset.copy(), r.junction_pos.copy(), r.vertex.copy(), r.strand.copy(),
            r.edges.copy(), plan.debug_candidates().copy(), plan.stats())


def same(a, b):
    for x, y in zip(a[:6], b[:6]):
        assert np.array_equal(x, y)


def same_junctions(a, b):
    # junction offsets, positions, vertices, strands, edges (not C1, which
    # depends on the filter)
    for x, y in zip(a[:5], b[:5]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("batch", [False, True])
def test_configs_do_not_change_results(batch):
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(5, n_sets=6, lo=20e3, hi=300e3)
    k, h = 31, 4
    if batch:
        plan = tp.Plan.batch([(to_genomes(c), tp.bloom_bits_for(to_genomes(c), k)) for c in sets],
                             k, h, BLOCKED)
    else:
        codes = [g for c in sets for g in c]
        plan = tp.Plan(to_genomes(codes), k, 2**24, h, BLOCKED)
    d_in = plan.upload()
    ref = outputs(plan, d_in)
    configs = [{"wg_per_cu": [1, 1, 1, 1]}, {"wg_per_cu": [2, 3, 4, 5]},
               {"tile_order": 1}, {"tile_order": 0, "wg_per_cu": [0, 0, 0, 0]},
               {"table_load": 16.0}, {"table_load": 0.05}, {"table_load": 4.0, "tile_order": 1},
               {"pass2_slabs": 1, "table_load": 0.7}, {"pass2_slabs": 2}, {"pass2_slabs": 3},
               {"pass2_slabs": 0}, {"pass2_slabs": 6}, {"pass2_slabs": 4, "fill_dedup": 0},
               {"fill_dedup": 1}, {"fill_dedup": 1, "tile_order": 1},
               {"fill_dedup": 1, "wg_per_cu": [1, 0, 0, 0]}, {"fill_dedup": 0},
               {"chunk_tiles": 2}, {"chunk_tiles": 5, "pass2_slabs": 1},
               {"chunk_tiles": 16, "pass2_slabs": 4, "fill_dedup": 0},
               {"chunk_tiles": 64, "tile_order": 1, "pass2_slabs": 3},
               {"tile_queue": 1, "chunk_tiles": 1, "tile_order": 0, "pass2_slabs": 2},
               {"tile_queue": 1, "chunk_tiles": 3, "pass2_slabs": 6},
               {"tile_queue": 1, "tile_order": 1, "pass2_slabs": 0},
               {"tile_queue": 1, "fill_dedup": 0, "wg_per_cu": [1, 1, 1, 1]},
               {"tile_queue": 1, "graphs": 1, "wg_per_cu": [0, 0, 6, 6]},
               {"tile_queue": 0, "graphs": 0}]
    for cfg in configs:
        say("case: config %s batch=%s" % (cfg, batch))
        plan.config = cfg
        got = outputs(plan, d_in)
        same(ref, got)
        if cfg.get("table_load") == 16.0:
            assert got[6]["table_attempts"] > 1  # the tables had to regrow
    plan.close()


def test_autotune_and_cache(tmp_path):
    import paper_1602_05856_amd as tp
    codes = synth.plain_small(2)
    cache = str(tmp_path / "tune.txt")
    plan = tp.Plan(to_genomes(codes), 25, 2**22, 3, BLOCKED)
    d_in = plan.upload()
    ref = outputs(plan, d_in)
    say("case: autotune plain_small")
    cfg = plan.autotune(d_in, cache)
    same(ref, outputs(plan, d_in))
    assert os.path.exists(cache)
    lines = [l for l in open(cache).read().splitlines() if l and not l.startswith("#")]
    assert len(lines) == 1 and len(lines[0].split()) == 14  # key + thirteen knobs
    # a second plan of the same shape takes the cached entry
    p2 = tp.Plan(to_genomes(codes), 25, 2**22, 3, BLOCKED)
    d2 = p2.upload()
    cfg2 = p2.autotune(d2, cache)
    assert cfg2["wg_per_cu"] == cfg["wg_per_cu"] and cfg2["tile_order"] == cfg["tile_order"]
    assert cfg2["table_load"] == pytest.approx(cfg["table_load"], abs=1e-3)
    for f in ("graphs", "pass2_slabs", "fill_dedup", "chunk_tiles", "bloom_bits_per_edge",
              "fill_binned", "tile_queue"):
        assert cfg2[f] == cfg[f], f
    with pytest.raises(tp.TwoPaCoError):
        p2.stats()  # a cache hit runs nothing
    same(ref, outputs(p2, d2))
    p2.close()
    plan.close()


@pytest.mark.parametrize("flags,k", [(BLOCKED, 25), (0, 31), (BLOCKED, 63), (BLOCKED, 100)])
def test_graph_replay_matches_direct_launches(flags, k):
    """Graphs on: every replay (with direct-launch runs and host waits in
    between, and a table regrowth that forces a new capture) gives the
    outputs of direct launches."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(61 + k, 3, 2000, 9000, alphabet=3, n_frac=0.001)
    plan = tp.Plan(to_genomes(codes), k, 2**16, 3, flags)
    d_in = plan.upload()
    ref = outputs(plan, d_in)
    plan.config = {"graphs": 1}
    for rep in range(4):
        say("case: graph replay %d k=%d flags=%d" % (rep, k, flags))
        got = outputs(plan, d_in)
        same(ref, got)
        assert got[6]["ms_fill"] > 0 and got[6]["ms_record"] > 0
        if rep == 1:
            plan.config = {"graphs": 0}
            same(ref, outputs(plan, d_in))  # direct launches between replays
            plan.config = {"graphs": 1}
        if rep == 2:
            plan.config = {"graphs": 1, "table_load": 16.0}  # regrowth: new pass-2 capture
    plan.config = {"graphs": 1, "table_load": 0.7}
    same(ref, outputs(plan, d_in))
    # the other table mode: new pass-2 captures with the any-size kernels,
    # replayed, then back to power-of-two tables
    for shape in (2, 2, 1):
        plan.config = {"graphs": 1, "table_shape": shape}
        same(ref, outputs(plan, d_in))
    plan.close()


def test_graphs_ignored_with_rounds():
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(71, 2, 2000, 5000, alphabet=3)
    plan = tp.Plan(to_genomes(codes), 25, 2**16, 3, BLOCKED)
    d_in = plan.upload()
    plan.rounds = 3
    ref = outputs(plan, d_in)
    plan.config = {"graphs": 1}
    same(ref, outputs(plan, d_in))
    plan.close()


def test_autotune_picks_filter_density_of_auto_sized_sets(tmp_path):
    """Sets created with bloom_bits 0: the tuner picks their density among 8,
    16 and 32 bits per (k+1)-mer, and every setting gives the same
    junctions, vertices, strands and edges."""
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(3, n_sets=12, lo=50e3, hi=2e6)
    plan = tp.Plan.batch([(to_genomes(c), 0) for c in sets], 31, 4, BLOCKED)
    d_in = plan.upload()
    ref = outputs(plan, d_in)
    for bpe in (8, 32):
        plan.config = {"bloom_bits_per_edge": bpe}
        got = outputs(plan, d_in)
        same_junctions(ref, got)
    say("case: autotune auto-sized batch")
    cfg = plan.autotune(d_in, str(tmp_path / "tune.txt"))
    assert cfg["bloom_bits_per_edge"] in (8, 16, 32)
    same_junctions(ref, outputs(plan, d_in))
    plan.close()
