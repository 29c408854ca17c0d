"""GPU parity of the batched form: many independent genome sets in one plan,
every phase one launch over all sets.  Each set's outputs (its Bloom filter,
candidates, junctions, vertex ids, strands, edges and counters) must equal
the oracle run on that set alone, and the plain one-set plan's outputs."""
import sys

import numpy as np
import pytest

import synth
from helpers import oracle_run, to_genomes

pytestmark = pytest.mark.gpu

SINGLE, PASS1, BLOCKED = 1, 2, 4


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


def run_batch(sets_codes, bs, k, h, flags, config=None):
    import paper_1602_05856_amd as tp
    plan = tp.Plan.batch([(to_genomes(c), b) for c, b in zip(sets_codes, bs)], k, h, flags)
    if config:
        plan.config = config
    d_in = plan.upload()
    plan.run(d_in)
    c1_all = plan.bitmap_positions(plan.debug_candidates())
    out = []
    for s in range(len(sets_codes)):
        g0 = plan.set_first_genome(s)
        out.append((plan.download(set_index=s), plan.debug_bloom(s),
                    c1_all[g0:g0 + len(sets_codes[s])], plan.stats(s)))
    total = plan.stats()
    whole = plan.download()
    plan.close()
    return out, total, whole


def edges_array(res):
    if not res.edges.size:
        return np.zeros((0, 3), np.uint64)
    return np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                     res.edges["to_pos"]], axis=1)


def check_set_vs_oracle(codes, got, k, b, h, flags, where):
    res, bloom, c1, st = got
    o, junctions, vx, edges = oracle_run(codes, k, b, h, flags)
    W = 1 if k <= 31 else (2 if k <= 63 else 4)
    assert np.array_equal(bloom, o.bloom), "Bloom words " + where
    for g in range(len(codes)):
        assert np.array_equal(c1[g], o.c1[g]), "C1 genome %d %s" % (g, where)
        assert np.array_equal(res.junctions(g), junctions[g]), "J genome %d %s" % (g, where)
        words, strand = vx[g]
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        assert np.array_equal(res.vertex[a:z, :W], words[:, :W]), "vertex genome %d %s" % (g, where)
        assert np.array_equal(res.strand[a:z], strand), "strand genome %d %s" % (g, where)
    assert np.array_equal(edges_array(res), edges.reshape(-1, 3)), "edges " + where
    assert st["candidates"] == o.stats["marks_pass1"], where
    assert st["junctions"] == sum(len(j) for j in junctions), where
    assert st["bloom_popcount"] == o.stats["bloom_popcount"], where
    assert st["positions"] == o.stats["positions"], where
    assert res.stats["junctions"] == st["junctions"], where


def mixed_sets(seed):
    """Uneven sets: empty, too short for k, N-split, tiny, and several tiles."""
    sets = [[],
            synth.random_genomes(seed, 2, 1, 20),
            synth.random_genomes(seed + 1, 3, 200, 3000, alphabet=2, n_frac=0.01),
            synth.random_genomes(seed + 2, 1, 5000, 9000, alphabet=3),
            [g[:20_000] for g in synth.plain_small(seed)[:3]],
            synth.random_genomes(seed + 3, 4, 0, 2500, alphabet=4, n_frac=0.002)]
    bs = [2**10, 2**6, 2**14, 2**8, 2**20, 2**12]
    return sets, bs


@pytest.mark.parametrize("k", [5, 25, 31, 40, 63, 100])
@pytest.mark.parametrize("flags", [0, BLOCKED, SINGLE, BLOCKED | PASS1])
def test_batch_sets_match_oracle(k, flags):
    sets, bs = mixed_sets(10 + k)
    say("case: batch mixed sets k=%d flags=%d" % (k, flags))
    got, total, whole = run_batch(sets, bs, k, 3, flags)
    for s, codes in enumerate(sets):
        check_set_vs_oracle(codes, got[s], k, bs[s], 3, flags, "set %d k=%d flags=%d" %
                            (s, k, flags))
    # batch totals and the whole download are the sets' concatenation
    assert total["junctions"] == sum(g[3]["junctions"] for g in got)
    assert total["candidates"] == sum(g[3]["candidates"] for g in got)
    assert whole.stats["junctions"] == total["junctions"]
    off = 0
    for s in range(len(sets)):
        res = got[s][0]
        n = res.junction_pos.size
        assert np.array_equal(whole.junction_pos[off:off + n], res.junction_pos)
        off += n


@pytest.mark.parametrize("k", [25, 40, 100])
@pytest.mark.parametrize("flags", [BLOCKED, BLOCKED | SINGLE])
def test_batch_binned_fill(k, flags):
    """The binned fill on a batch: every set's items land in its own part of
    the filter pool (one set of 2^28 bits spans two buckets; others are
    empty or too short for k), in chunks of 2 tiles; every set equals the
    oracle."""
    sets, bs = mixed_sets(40 + k)
    bs[4] = 2**28
    say("case: batch binned fill k=%d flags=%d" % (k, flags))
    got, total, _ = run_batch(sets, bs, k, 3, flags,
                              config={"fill_binned": 2, "bin_chunk_tiles": 2})
    for s, codes in enumerate(sets):
        check_set_vs_oracle(codes, got[s], k, bs[s], 3, flags, "set %d k=%d flags=%d" %
                            (s, k, flags))


@pytest.mark.parametrize("bpe", [8, 16, 32])
def test_batch_auto_sized_filters(bpe):
    """Sets created with bloom_bits 0, sized by the plan at bpe bits per
    (k+1)-mer: every set equals the oracle run with the size it got."""
    sets, _ = mixed_sets(70 + bpe)
    k = 25
    say("case: batch of auto-sized filters at %d bits per edge" % bpe)
    got, total, _ = run_batch(sets, [0] * len(sets), k, 3, BLOCKED,
                              config={"bloom_bits_per_edge": bpe})
    for s, codes in enumerate(sets):
        b = got[s][1].size * 32
        check_set_vs_oracle(codes, got[s], k, b, 3, BLOCKED, "auto set %d bpe %d" % (s, bpe))


@pytest.mark.parametrize("k", [25, 40, 100])
def test_batch_any_size_tables(k):
    # the any-size table mode with several set tables in one pool, one of
    # them regrowing (load target 8 against the candidate count)
    sets, bs = mixed_sets(40 + k)
    say("case: batch any-size tables k=%d" % k)
    got, total, _ = run_batch(sets, bs, k, 3, BLOCKED, config={"table_shape": 2, "table_load": 8.0})
    for s, codes in enumerate(sets):
        check_set_vs_oracle(codes, got[s], k, bs[s], 3, BLOCKED, "set %d k=%d any-size" % (s, k))
    assert total["table_attempts"] > 1
    # the plan's table is its sets' tables, each with its 4096-slot spare tail
    caps = [g[3]["table_capacity"] for g in got]
    assert total["table_capacity"] == sum(caps)
    assert all(c >= 1024 + 4096 and (c - 4096) % 64 == 0 for c in caps), caps


@pytest.mark.parametrize("flags", [0, BLOCKED])
def test_batch_equals_alone(flags):
    """Every set gives the same outputs in a batch as in a plan of its own."""
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(1, n_sets=12, lo=20e3, hi=400e3)
    k, h = 31, 4
    bs = [tp.bloom_bits_for(to_genomes(c), k) for c in sets]
    say("case: batch vs alone, 12 sets, flags=%d" % flags)
    got, _, _ = run_batch(sets, bs, k, h, flags)
    for s, codes in enumerate(sets):
        plan = tp.Plan(to_genomes(codes), k, bs[s], h, flags)
        d_in = plan.upload()
        plan.run(d_in)
        alone = plan.download()
        bloom = plan.debug_bloom()
        c1 = plan.bitmap_positions(plan.debug_candidates())
        st = plan.stats()
        plan.close()
        res, bbloom, bc1, bst = got[s]
        assert np.array_equal(bbloom, bloom), "set %d bloom" % s
        for g in range(len(codes)):
            assert np.array_equal(bc1[g], c1[g]), "set %d C1 genome %d" % (s, g)
        for f in ("junction_offset", "junction_pos", "vertex", "strand"):
            assert np.array_equal(getattr(res, f), getattr(alone, f)), "set %d %s" % (s, f)
        assert np.array_equal(res.edges, alone.edges), "set %d edges" % s
        for f in ("positions", "candidates", "junctions", "edges", "bloom_popcount"):
            assert bst[f] == st[f], "set %d %s" % (s, f)


def test_batch_config3_shape_sample():
    """Sets drawn as in the batched workload (k=31, 16 bits per (k+1)-mer,
    h=4), at reduced sizes so that the oracle checks every set."""
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(2, n_sets=24, lo=50e3, hi=1e6)
    k, h = 31, 4
    bs = [tp.bloom_bits_for(to_genomes(c), k) for c in sets]
    say("case: batched workload sample, 24 sets, %.1f Mbp" %
        (sum(g.size for c in sets for g in c) / 1e6))
    got, _, _ = run_batch(sets, bs, k, h, BLOCKED)
    for s, codes in enumerate(sets):
        check_set_vs_oracle(codes, got[s], k, bs[s], h, BLOCKED, "config3 set %d" % s)


def test_batch_rerun_is_deterministic():
    import paper_1602_05856_amd as tp
    sets, bs = mixed_sets(3)
    plan = tp.Plan.batch([(to_genomes(c), b) for c, b in zip(sets, bs)], 25, 3, BLOCKED)
    d_in = plan.upload()
    outs = []
    for _ in range(3):
        plan.run(d_in)
        r = plan.download()
        outs.append((r.junction_pos.copy(), edges_array(r).copy(), plan.stats()["candidates"]))
    plan.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert o[2] == outs[0][2]


@pytest.mark.parametrize("dedup", [0, 1])
def test_batch_identical_sets_fill_dedup(dedup):
    """Identical sets side by side: a filter effect (block, offset, stride,
    pair) sent for one set's filter must not count for the next set's, so
    every set's filter equals the oracle's with the fill's dedup on."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(77, 3, 3000, 7000, alphabet=4)
    k, h, b = 21, 3, 2**12
    sets = [codes] * 5
    plan = tp.Plan.batch([(to_genomes(c), b) for c in sets], k, h, BLOCKED)
    plan.config = {"fill_dedup": dedup}
    say("case: identical sets, fill_dedup=%d" % dedup)
    d_in = plan.upload()
    plan.run(d_in)
    o, junctions, _, _ = oracle_run(codes, k, b, h, BLOCKED)
    for s in range(len(sets)):
        assert np.array_equal(plan.debug_bloom(s), o.bloom), "set %d" % s
        st = plan.stats(s)
        assert st["candidates"] == o.stats["marks_pass1"], "set %d" % s
        assert st["junctions"] == sum(len(j) for j in junctions), "set %d" % s
        res = plan.download(set_index=s)
        for g in range(len(codes)):
            assert np.array_equal(res.junctions(g), junctions[g]), "set %d genome %d" % (s, g)
    assert len({plan.stats(s)["table_keys"] for s in range(len(sets))}) == 1
    plan.close()


def test_batched_workload_full_size_digests():
    """The full batched workload (256 sets, ~846 Mbp, k = 31, h = 4, blocked
    filter at 16 bits per (k+1)-mer) in the configuration the autotuner picks
    (as bench.py times it), and on caller memory (the graph-capturable run):
    every set's filter, candidates, junctions, vertices, strands and edges
    against the digests of the oracle run on that set alone
    (tests/golden/batched_k31_blocked.json, written by
    make_batched_digests.py from the oracle only)."""
    import json
    import os

    import torch

    import paper_1602_05856_amd as tp
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    from digests import digest_outputs
    rec = json.load(open(os.path.join(here, "golden", "batched_k31_blocked.json")))
    k, h = rec["k"], rec["hashes"]
    sets = synth.batched_sets(0, n_sets=len(rec["sets"]))
    gsets = [to_genomes(c) for c in sets]
    bs = [tp.bloom_bits_for(g, k) for g in gsets]
    assert bs == [r["bloom_bits"] for r in rec["sets"]], "filter sizes differ from the oracle's"
    plan = tp.Plan.batch(list(zip(gsets, bs)), k, h, BLOCKED)
    d_in = plan.upload()
    say("case: batched workload full size, %d sets; tuned %s" % (len(sets), plan.autotune(d_in)))
    plan.run(d_in)
    c1_all = plan.bitmap_positions(plan.debug_candidates())
    for s, (codes, want) in enumerate(zip(sets, rec["sets"])):
        res = plan.download(set_index=s)
        g0 = plan.set_first_genome(s)
        ng = len(codes)
        vertex = [res.vertex[res.junction_offset[g]:res.junction_offset[g + 1]]
                  for g in range(ng)]
        strand = [res.strand[res.junction_offset[g]:res.junction_offset[g + 1]]
                  for g in range(ng)]
        got = digest_outputs(plan.debug_bloom(s), c1_all[g0:g0 + ng],
                             [res.junctions(g) for g in range(ng)], vertex, strand,
                             edges_array(res), 1)
        assert got["counts"] == want["counts"], s
        for key in ("bloom", "c1", "junctions", "vertex", "strand", "edges"):
            assert got[key] == want[key], (s, key)
    # the same batch on caller memory, captured once as a graph and replayed
    plan.workspace_layout(0.25, 0.25)
    ws, out = plan.alloc_workspace()
    plan.prepare_workspace(ws)
    s_ = torch.cuda.Stream()
    s_.wait_stream(torch.cuda.current_stream())
    g_ = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s_):
        plan.run_ws(d_in, ws, out, stream=s_)
        s_.synchronize()
        with torch.cuda.graph(g_, stream=s_):
            plan.run_ws(d_in, ws, out, stream=s_)
    torch.cuda.current_stream().wait_stream(s_)
    out.fill_(0)
    g_.replay()
    torch.cuda.synchronize()
    cnt = plan.ws_counts(out)
    assert cnt["status"] == 0, cnt
    res = plan.ws_result(out)
    all_edges = edges_array(res)
    g0 = 0
    for s, (codes, want) in enumerate(zip(sets, rec["sets"])):
        ng = len(codes)
        js = [res.junctions(g0 + g) for g in range(ng)]
        sel = (all_edges[:, 0] >= g0) & (all_edges[:, 0] < g0 + ng)
        e = all_edges[sel].copy()
        e[:, 0] -= np.uint64(g0)
        got = digest_outputs(np.zeros(1, np.uint32), [[]] * ng, js,
                             [res.vertex[res.junction_offset[g0 + g]:
                                         res.junction_offset[g0 + g + 1]] for g in range(ng)],
                             [res.strand[res.junction_offset[g0 + g]:
                                         res.junction_offset[g0 + g + 1]] for g in range(ng)],
                             e, 1)
        for key in ("junctions", "vertex", "strand", "edges"):
            assert got[key] == want[key], (s, key)
        g0 += ng
    del g_
    plan.close()
