"""GPU parity of Algorithm 3 (multiple rounds): against the oracle's rounds
run, bit-exact -- class bounds, the last round's filter, the union of the
rounds' candidates, junctions, vertices, strands, edges and counters -- and
the junction outputs of the full-size workload against the stored
single-round digests (junctions do not depend on the number of rounds)."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import to_genomes

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from digests import digest_outputs  # noqa: E402

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


def edges_of(res):
    if not res.edges.size:
        return np.zeros((0, 3), np.uint64)
    return np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                     res.edges["to_pos"]], axis=1)


def check_rounds(plan, set_index, codes, k, b, h, l, flags, where):
    single = bool(flags & SINGLE)
    o = oracle.rounds(codes, k, b, h, l, single_strand=single, blocked=bool(flags & BLOCKED))
    junctions = o.c1 if flags & PASS1 else o.junctions
    res = plan.download(set_index=set_index)
    st = plan.stats(set_index)
    g0 = plan.set_first_genome(set_index)
    c1 = plan.bitmap_positions(plan.debug_candidates())[g0:g0 + len(codes)]
    assert np.array_equal(plan.class_bounds(set_index), o.bounds), "bounds " + where
    assert np.array_equal(plan.debug_bloom(set_index), o.bloom), "last filter " + where
    for g in range(len(codes)):
        assert np.array_equal(c1[g], o.c1[g]), "C1 union, genome %d %s" % (g, where)
        assert np.array_equal(res.junctions(g), junctions[g]), "J, genome %d %s" % (g, where)
        words, strand = oracle.vertex_words(codes[g], k, junctions[g], single_strand=single)
        W = 1 if k <= 31 else (2 if k <= 63 else 4)
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        assert np.array_equal(res.vertex[a:z, :W], words[:, :W]), "vertex, genome %d %s" % (g, where)
        assert np.array_equal(res.strand[a:z], strand), "strand %s" % where
    assert np.array_equal(edges_of(res), oracle.edges(codes, k, junctions).reshape(-1, 3)), where
    assert st["candidates"] == o.stats["marks_pass1"], where
    assert st["bloom_popcount"] == o.stats["bloom_popcount"], where
    assert st["junctions"] == sum(len(j) for j in junctions), where


@pytest.mark.parametrize("k", [5, 25, 31, 40, 63, 100])
@pytest.mark.parametrize("flags", [0, BLOCKED, SINGLE | BLOCKED, PASS1 | BLOCKED])
def test_rounds_match_oracle(k, flags):
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(500 + k, 3, 1000, 6000, alphabet=3, n_frac=0.002)
    codes += [synth.plain_small(2)[1][:9000]]
    b, h = 2**15, 3
    plan = tp.Plan(to_genomes(codes), k, b, h, flags)
    d_in = plan.upload()
    for l in (1, 2, 3, 8):
        say("case: rounds k=%d flags=%d l=%d" % (k, flags, l))
        plan.rounds = l
        plan.run(d_in)
        check_rounds(plan, 0, codes, k, b, h, l, flags, "k=%d flags=%d l=%d" % (k, flags, l))
    plan.close()


@pytest.mark.parametrize("k", [25, 63])
def test_rounds_with_tile_queue(k):
    """Rounds with the tile kernels taking their chunks from device queues
    (cleared before every round and every second-pass attempt)."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(900 + k, 3, 1000, 6000, alphabet=3, n_frac=0.002)
    codes += [synth.plain_small(5)[1][:9000]]
    b, h = 2**15, 3
    plan = tp.Plan(to_genomes(codes), k, b, h, BLOCKED)
    plan.config = {"tile_queue": 1, "chunk_tiles": 2, "table_load": 8.0}
    d_in = plan.upload()
    for l in (1, 3):
        say("case: rounds with tile queue k=%d l=%d" % (k, l))
        plan.rounds = l
        plan.run(d_in)
        check_rounds(plan, 0, codes, k, b, h, l, BLOCKED, "queue k=%d l=%d" % (k, l))
    plan.close()


@pytest.mark.parametrize("k", [25, 63])
def test_rounds_binned_fill(k):
    """Rounds with the binned fill: each round's filter holds only the edges
    next to a k-mer of its class, built in chunks of 1 tile."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(700 + k, 3, 1000, 6000, alphabet=3, n_frac=0.002)
    codes += [synth.plain_small(4)[1][:9000]]
    b, h = 2**24, 3
    plan = tp.Plan(to_genomes(codes), k, b, h, BLOCKED)
    plan.config = {"fill_binned": 2, "bin_chunk_tiles": 1}
    d_in = plan.upload()
    for l in (1, 3):
        say("case: rounds binned k=%d l=%d" % (k, l))
        plan.rounds = l
        plan.run(d_in)
        check_rounds(plan, 0, codes, k, b, h, l, BLOCKED, "binned k=%d l=%d" % (k, l))
    plan.close()


@pytest.mark.parametrize("k", [16, 25])
def test_rounds_binned_record(k):
    """Rounds with the binned record: each round's table (its class's
    candidate k-mers) built block by block, in two passes; a small filter
    makes most positions candidates."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(900 + k, 3, 2000, 30000, alphabet=3, n_frac=0.002)
    b, h = 2**14, 3
    plan = tp.Plan(to_genomes(codes), k, b, h, BLOCKED)
    plan.config = {"record_binned": 2, "table_shape": 2, "record_passes": 2}
    d_in = plan.upload()
    for l in (1, 3):
        say("case: rounds, binned record k=%d l=%d" % (k, l))
        plan.rounds = l
        plan.run(d_in)
        assert plan.stats()["record_passes"] >= 1
        check_rounds(plan, 0, codes, k, b, h, l, BLOCKED, "binned record k=%d l=%d" % (k, l))
    plan.close()


def test_binned_record_needs_one_set():
    """A batch records directly whatever record_binned asks (its items
    would not say which set's table they belong to)."""
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(11, n_sets=3, lo=20e3, hi=100e3)
    k, h = 25, 3
    bs = [2**14] * len(sets)
    plan = tp.Plan.batch([(to_genomes(c), b) for c, b in zip(sets, bs)], k, h, BLOCKED)
    plan.config = {"record_binned": 2, "table_shape": 2}
    d_in = plan.upload()
    say("case: binned record asked for a batch of %d sets" % len(sets))
    plan.run(d_in)
    assert plan.stats()["record_passes"] == 0
    for s, codes in enumerate(sets):
        check_rounds(plan, s, codes, k, bs[s], h, 1, BLOCKED, "set %d" % s)
    plan.close()


def test_rounds_in_a_batch():
    import paper_1602_05856_amd as tp
    sets = synth.batched_sets(9, n_sets=6, lo=20e3, hi=300e3) + [[], synth.random_genomes(3, 2, 1, 20)]
    k, h = 31, 4
    bs = [tp.bloom_bits_for(to_genomes(c), k) if c else 2**10 for c in sets]
    plan = tp.Plan.batch([(to_genomes(c), b) for c, b in zip(sets, bs)], k, h, BLOCKED)
    d_in = plan.upload()
    plan.rounds = 4
    say("case: rounds in a batch of %d sets" % len(sets))
    plan.run(d_in)
    for s, codes in enumerate(sets):
        check_rounds(plan, s, codes, k, bs[s], h, 4, BLOCKED, "set %d" % s)
    plan.close()


@pytest.mark.parametrize("case", ["bacterial_k25_blocked.json", "bacterial_k63.json"])
def test_rounds_full_size_junctions(case):
    import paper_1602_05856_amd as tp
    path = os.path.join(HERE, "golden", case)
    if not os.path.exists(path):
        pytest.skip("oracle digests %s not generated" % case)
    rec = json.load(open(path))
    k = rec["k"]
    W = 1 if k <= 31 else 2
    flags = tp.TP_FLAG_BLOCKED_FILTER if rec.get("filter") == "blocked" else 0
    codes = synth.bacterial(0)
    plan = tp.Plan(to_genomes(codes), k, 1 << rec["bloom_log2"], rec["hashes"], flags)
    d_in = plan.upload()
    plan.rounds = 4
    say("case: full-size %s with 4 rounds" % case)
    plan.run(d_in)
    res = plan.download()
    plan.close()
    ng = len(codes)
    junctions = [res.junctions(g) for g in range(ng)]
    vertex, strand = [], []
    for g in range(ng):
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        v = np.zeros((z - a, 2), np.uint64)
        v[:, :W] = res.vertex[a:z]
        vertex.append(v)
        strand.append(res.strand[a:z])
    got = digest_outputs(np.zeros(1, np.uint32), [np.zeros(0, np.uint64)] * ng, junctions,
                         vertex, strand, edges_of(res), W)
    for key in ("junctions", "vertex", "strand", "edges"):
        assert got[key] == rec[key], key
    assert got["counts"]["junctions"] == rec["counts"]["junctions"]


@pytest.mark.parametrize("k, flags", [(25, BLOCKED), (33, 0)])
def test_table_budget_forces_rounds(k, flags):
    """A table budget below the one-round exact table makes the run take
    Algorithm 3 with enough rounds: every output equals the oracle's
    Algorithm 3 with that many rounds, and the junctions those of one round."""
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(620 + k, 3, 3000, 9000, alphabet=3, n_frac=0.002)
    b, h = 2**15, 3
    plan = tp.Plan(to_genomes(codes), k, b, h, flags)
    d_in = plan.upload()
    plan.run(d_in)
    one = plan.stats()
    assert one["rounds"] == 1
    want_j = [plan.download().junctions(g).copy() for g in range(len(codes))]
    slot_bytes = 8 if k <= 27 else (9 if k <= 31 else 16)
    budget = one["table_capacity"] * slot_bytes // 3
    plan.config = {"table_budget": budget}
    say("case: table budget %d bytes, k=%d flags=%d" % (budget, k, flags))
    plan.run(d_in)
    st = plan.stats()
    l = st["rounds"]
    assert l >= 3, st
    assert len(plan.class_bounds(0)) == l + 1
    check_rounds(plan, 0, codes, k, b, h, l, flags, "budget k=%d l=%d" % (k, l))
    res = plan.download()
    for g in range(len(codes)):
        assert np.array_equal(res.junctions(g), want_j[g])
    # a budget the one-round table fits keeps one round
    plan.config = {"table_budget": one["table_capacity"] * slot_bytes * 4}
    plan.run(d_in)
    assert plan.stats()["rounds"] == 1
    plan.close()
