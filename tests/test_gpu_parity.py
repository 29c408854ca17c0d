"""GPU parity: the library's HIP path against the CPU oracle, element by
element, on seeded inputs.  Everything here is integer work, so the bar is
bit-exact: Bloom filter words, the first-pass candidate bitmap, junction
positions, vertex ids, strands, edges and counters."""
import sys

import numpy as np
import pytest

import synth
from helpers import assert_parity, gpu_run, oracle_run

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


@pytest.mark.parametrize("flags", [0, BLOCKED])
def test_plain_small_full_parity(flags):
    # 4 x 100 kbp, k=25, b=2^24, h=3: many tiles per genome, ragged tails
    gs = synth.plain_small(0)
    say("case: plain_small k=25 b=2^24 h=3 flags=%d" % flags)
    res, o = assert_parity(gs, 25, 2**24, 3, flags=flags, label="plain_small")
    assert res.stats["junctions"] > 1000


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 16, 24, 25, 30, 31, 32, 33, 48, 62, 63,
                               64, 65, 80, 96, 100, 127])
def test_k_sweep(k):
    # low-complexity genomes so that junctions are plentiful at every k
    gs = synth.random_genomes(100 + k, 3, 1000, 6000, alphabet=2)
    gs += [synth.plain_small(1)[0][:7000]]
    for b, h, flags in ((2**14, 4, 0), (2**22, 2, 0), (2**14, 4, BLOCKED), (2**20, 3, BLOCKED)):
        say("case: k_sweep k=%d b=%d h=%d flags=%d" % (k, b, h, flags))
        assert_parity(gs, k, b, h, flags=flags, label="k_sweep")


@pytest.mark.parametrize("flags", [SINGLE, PASS1, SINGLE | PASS1, BLOCKED | SINGLE,
                                   BLOCKED | PASS1])
def test_flags(flags):
    gs = synth.random_genomes(7, 4, 500, 5000, alphabet=3, n_frac=0.01)
    for k in (5, 25, 40):
        say("case: flags=%d k=%d" % (flags, k))
        assert_parity(gs, k, 2**16, 3, flags=flags, label="flags")


def test_random_tiny_cases():
    r = np.random.default_rng(2024)
    for case in range(120):
        n = int(r.integers(1, 7))
        gs = synth.random_genomes(5000 + case, n, 0, int(r.choice([40, 300, 3000])),
                                  alphabet=int(r.integers(1, 5)),
                                  n_frac=float(r.choice([0.0, 0.02, 0.2])))
        k = int(r.integers(1, 64))
        b = int(2 ** r.integers(6, 20))
        h = int(r.integers(1, 17))
        flags = int(r.choice([0, 0, SINGLE, PASS1, BLOCKED, BLOCKED, BLOCKED | SINGLE]))
        say("case: tiny %d n=%d k=%d b=%d h=%d flags=%d" % (case, n, k, b, h, flags))
        assert_parity(gs, k, b, h, flags=flags, label="tiny%d" % case)


def test_edge_lengths_and_empty():
    k = 11
    A = synth.random_bases(synth.rng(77, 1), 4000)
    gs = [np.zeros(0, np.uint8), A[:k - 1], A[:k], A[:k + 1], A[:k + 2],
          np.full(50, 4, np.uint8), A[:2048], A[:2049], A[:4000]]
    for flags in (0, BLOCKED):
        say("case: edge lengths flags=%d" % flags)
        assert_parity(gs, k, 2**12, 3, flags=flags, label="edge-lengths")
    say("case: no genomes")
    plan, res, bloom, c1 = gpu_run([], k, 2**10, 2)
    assert res.stats["junctions"] == 0 and res.edges.size == 0
    assert list(res.junction_offset) == [0]


def test_homopolymer_and_many_strings():
    k = 4
    homo = np.zeros(5000, np.uint8)
    # N every 7 bases: thousands of short strings per tile
    chopped = synth.random_bases(synth.rng(78, 1), 20000)
    chopped[::7] = 4
    for flags in (0, BLOCKED):
        say("case: homopolymer + chopped flags=%d" % flags)
        res, _ = assert_parity([homo, chopped], k, 2**12, 2, flags=flags, label="homo")
        assert res.junctions(0).size == 5000 - k + 1


def test_saturated_filter_and_many_hashes():
    gs = synth.random_genomes(31, 3, 2000, 4000, alphabet=4)
    for b, h, flags in ((32, 16, 0), (64, 1, 0), (2**10, 16, 0), (64, 16, BLOCKED),
                        (128, 3, BLOCKED)):
        say("case: saturated b=%d h=%d flags=%d" % (b, h, flags))
        assert_parity(gs, 13, b, h, flags=flags, label="saturated")


def test_repeat_runs_are_deterministic():
    gs = synth.plain_small(2)
    plan, res1, bloom1, c11 = gpu_run(gs, 25, 2**20, 3)
    d_in = plan.upload()
    for _ in range(3):
        plan.run(d_in)
        res2 = plan.download()
        assert np.array_equal(res1.junction_pos, res2.junction_pos)
        assert np.array_equal(res1.vertex, res2.vertex)
        assert np.array_equal(res1.edges, res2.edges)
        assert np.array_equal(bloom1, plan.debug_bloom())
    plan.close()


def test_host_build_matches_device_path():
    import paper_1602_05856_amd as tp
    from helpers import to_genomes
    gs = synth.random_genomes(41, 3, 3000, 9000, alphabet=3, n_frac=0.001)
    res = tp.twopaco_build(to_genomes(gs), 21, 2**18, 4)
    o, junctions, vx, edges = oracle_run(gs, 21, 2**18, 4)
    for g in range(len(gs)):
        assert np.array_equal(res.junctions(g), junctions[g])


def test_two_word_keys_repeated_within_a_wave():
    # k >= 32: many lanes of one wave insert the same new two-word key (a
    # homopolymer, a short tandem repeat); the claimer must publish while its
    # wave-mates wait on the pending high word
    rep = np.tile(synth.random_bases(synth.rng(79, 1), 7), 900)
    homo = np.full(3000, 2, np.uint8)
    for k in (32, 40, 55, 63, 64, 100, 127):
        for flags in (0, BLOCKED):
            say("case: repeated multi-word keys k=%d flags=%d" % (k, flags))
            assert_parity([homo, rep], k, 2**12, 3, flags=flags, label="rep2w")


@pytest.mark.parametrize("flags", [0, BLOCKED, SINGLE, PASS1 | BLOCKED, SINGLE | BLOCKED])
def test_four_word_kmers(flags):
    # k = 64..127 (four-word values): random and low-complexity genomes with N
    # stretches, strings around k long, several tiles
    gs = synth.random_genomes(7100 + flags, 4, 100, 6000, alphabet=2, n_frac=0.0005)
    gs += [np.full(700, 1, np.uint8), synth.random_genomes(7200, 1, 5000, 5000)[0],
           synth.random_genomes(7300, 1, 128, 128)[0]]
    for k in (64, 90, 100, 127):
        say("case: four-word k=%d flags=%d" % (k, flags))
        assert_parity(gs, k, 2**14, 3, flags=flags, label="w4")


@pytest.mark.parametrize("k", [5, 25, 40, 100])
def test_strings_cut_at_lane_run_and_tile_boundaries(k):
    """The blocked query carries a position's in-middle key from the lane
    below, lane 63 into the next step's lane 0, and computes it afresh at the
    start of each wave's 512-position run; strings starting or ending exactly
    at those offsets (and at tile boundaries) must still match the oracle."""
    base = synth.random_bases(synth.rng(79, k), 3 * 2048 + 500)
    g = base.copy()
    # an N at offset c ends one string at c and starts the next at c + 1
    for c in (63, 127, 128, 511, 512, 1023, 2047, 2048 + 64, 2048 + 511, 2 * 2048 - 1,
              2 * 2048 + 512 + 63):
        g[c] = 4
    related = g.copy()
    snp = synth.rng(79, k, 1).integers(0, related.size, 40)
    related[snp] = (related[snp] + 1) % 4
    related[g == 4] = 4
    for flags in (0, BLOCKED):
        say("case: boundary strings k=%d flags=%d" % (k, flags))
        assert_parity([g, related, base[:2048 + 63]], k, 2**14, 3, flags=flags,
                      label="boundaries")


@pytest.mark.parametrize("k", [5, 25, 31, 40, 63, 100])
@pytest.mark.parametrize("shape", [1, 2])
def test_table_shapes(k, shape):
    # both exact-table modes (power of two with wrapping probes; any size in
    # blocks of 8192 slots, probes wrapping within a block), each at a normal
    # load and at a load target that overflows the table so that it regrows
    # (doubling keeps the any-size capacity in whole blocks)
    gs = synth.random_genomes(300 + k, 3, 1000, 8000, alphabet=3, n_frac=0.005)
    gs += [synth.plain_small(2)[0][:9000]]
    for load, flags in ((0.7, 0), (8.0, BLOCKED)):
        cfg = {"table_shape": shape, "table_load": load}
        say("case: table_shape=%d load=%.1f k=%d flags=%d" % (shape, load, k, flags))
        res, _ = assert_parity(gs, k, 2**16, 3, flags=flags, label="table_shape", config=cfg)
        st = res.stats
        home = st["table_capacity"] - 4096  # slots past the spare tail
        assert home % 64 == 0
        if shape == 1 or home <= 8192:
            assert home & (home - 1) == 0, home
        else:
            assert home % 8192 == 0, home
        if load > 1 and k >= 25:  # k = 5 has at most 512 keys: the smallest table holds them
            assert st["table_attempts"] > 1


@pytest.mark.parametrize("k", [4, 16, 25, 27])
def test_binned_record(k):
    # the binned record (candidates partitioned by home block of the table,
    # each block built in LDS) against the oracle: any-size tables of several
    # blocks in one pass and in 3 passes, a power-of-two table (binned only
    # while it is one block), single strand, and a load target that
    # overflows the blocks so that the table doubles; a small filter makes
    # most positions candidates
    gs = synth.random_genomes(800 + k, 3, 1000, 40000, alphabet=3, n_frac=0.005)
    gs += [synth.plain_small(3)[0][:30000]]
    for shape, load, passes, flags in ((2, 0.7, 0, BLOCKED), (2, 0.7, 3, 0),
                                       (1, 0.7, 0, BLOCKED | SINGLE), (2, 8.0, 2, BLOCKED)):
        cfg = {"record_binned": 2, "table_shape": shape, "table_load": load,
               "record_passes": passes}
        say("case: binned record k=%d shape=%d load=%.1f passes=%d flags=%d" % (
            k, shape, load, passes, flags))
        res, _ = assert_parity(gs, k, 2**14, 3, flags=flags, label="binned record", config=cfg)
        st = res.stats
        home = st["table_capacity"] - 4096
        if shape == 2 or home <= 8192:
            # blocks of 8192 slots (or one smaller block), split evenly over
            # the passes asked for
            nblk = max(1, home // 8192)
            per = -(-nblk // max(1, passes))
            assert st["record_passes"] == -(-nblk // per), st
        else:
            assert st["record_passes"] == 0, st
        if load > 1 and k >= 16:
            assert st["table_attempts"] > 1


@pytest.mark.parametrize("k", [5, 25, 31, 40, 63, 100])
def test_binned_fill(k):
    # the binned fill (edge items partitioned by filter region, applied in
    # LDS) against the oracle: one chunk; chunks of 1 and 3 tiles, so that
    # regions are read back between chunks; 2^28 bits = 2 buckets of 256
    # regions; h = 5; single strand; first pass only
    gs = synth.random_genomes(500 + k, 3, 1000, 9000, alphabet=3, n_frac=0.005)
    gs += [synth.plain_small(3)[0][:30000]]
    for b, h, chunk, flags in ((2**20, 3, 0, BLOCKED), (2**28, 3, 1, BLOCKED),
                               (2**28, 5, 3, BLOCKED | SINGLE), (2**16, 4, 2, BLOCKED | PASS1)):
        cfg = {"fill_binned": 2, "bin_chunk_tiles": chunk}
        say("case: binned fill k=%d b=%d h=%d chunk=%d flags=%d" % (k, b, h, chunk, flags))
        res, _ = assert_parity(gs, k, b, h, flags=flags, label="binned", config=cfg)
        assert res.stats["fill_atomics"] > 0
