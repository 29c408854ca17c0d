"""Pins for the CPU oracle against facts that do not come from the oracle
itself: published test vectors, the worked example of Fig. 1 derived from the
definitions, closed forms, invariants stated in the paper, and the
false-positive analysis of the Theoretical Analysis section."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = 2**64


def enc(s):
    return np.array(["ACGTN".index(ch) for ch in s], dtype=np.uint8)


def as_sets(lists):
    return [set(int(x) for x in l) for l in lists]


# ------------------------------------------------------------------ hash spec

def test_mix64_matches_published_splitmix64_vectors():
    golden = 0x9E3779B97F4A7C15
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_vectors.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for seed, i, want in rows:
        state = (int(seed) + int(i) * golden) % M64
        assert oracle.mix64(state) == int(want, 0)


@pytest.mark.parametrize("k", [5, 25, 31, 32, 63])
def test_bloom_indices_are_a_progression_of_distinct_bits(k):
    # double hashing: idx_t = H1 + t*H2 mod b with H2 odd, so for b = 2^B the h
    # indices are distinct and consecutive differences are constant mod b.
    r = np.random.default_rng(k)
    for _ in range(200):
        v = int(r.integers(0, 2**63)) | (int(r.integers(0, 2**62)) << 64 if k >= 32 else 0)
        v &= (1 << (2 * (k + 1))) - 1
        for b in (2**10, 2**24):
            idx = oracle.bloom_indices(v, k, b, 8)
            assert len(set(idx)) == 8
            d = {(idx[t + 1] - idx[t]) % b for t in range(7)}
            assert len(d) == 1 and d.pop() % 2 == 1
            assert all(0 <= x < b for x in idx)


# ----------------------------------------------------- worked example, Fig. 1

def _fig1_rows():
    rows = []
    for line in open(os.path.join(GOLDEN, "fig1_example.txt")):
        if line.strip() and not line.startswith("#"):
            mode, s, js, es = line.split()
            rows.append((mode, s, [int(x) for x in js.split(",")],
                         [tuple(int(y) for y in e.split("-")) for e in es.split(",")]))
    return rows


@pytest.mark.parametrize("mode", ["single", "both"])
def test_fig1_worked_example(mode):
    rows = [r for r in _fig1_rows() if r[0] == mode]
    genomes = [enc(r[1]) for r in rows]
    single = mode == "single"
    bf = oracle.bruteforce(genomes, 2, single_strand=single)
    tp = oracle.twopass(genomes, 2, 2**16, 3, single_strand=single)
    for (m, s, want_j, want_e), got_bf, got_tp in zip(rows, bf, tp.junctions):
        assert list(got_bf) == want_j
        assert list(got_tp) == want_j
    e = oracle.edges(genomes, 2, tp.junctions)
    for gi, (m, s, want_j, want_e) in enumerate(rows):
        got = [(int(a), int(b)) for g, a, b in e if g == gi]
        assert got == want_e


def test_fig1_false_edge_makes_gc_a_candidate():
    # Fig. 1(d): with a Bloom filter, a false edge can leave GC (position 2)
    # marked after the first pass; the second pass always removes it.  Small,
    # crowded filters make such false edges likely.
    genomes = [enc("TGGCACGTC"), enc("TGGCACTTC")]
    seen = False
    for b in (32, 64):
        for h in range(1, 9):
            tp = oracle.twopass(genomes, 2, b, h, single_strand=True)
            seen |= 2 in set(int(x) for x in tp.c1[0])
            assert list(tp.junctions[0]) == [0, 4, 7]
            assert list(tp.junctions[1]) == [0, 4, 7]
    assert seen


def _bases(mask_text):
    return 0 if mask_text == "-" else sum(1 << "ACGT".index(ch) for ch in mask_text)


def _value(text):
    v = 0
    for ch in text:
        v = 4 * v + "ACGT".index(ch)
    return v


@pytest.mark.parametrize("mode", ["single", "both"])
def test_fig1_vertex_masks(mode):
    # in/out edges of every vertex of the Fig. 1 graph, derived by hand
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fig1_masks.txt"))
            if l.strip() and not l.startswith("#")]
    rows = [r for r in rows if r[0] == mode]
    assert rows
    genomes = [enc("TGGCACGTC"), enc("TGGCACTTC")]
    single = mode == "single"
    for threads in (1, 3):
        inm, outm, sent = oracle.vertex_masks(genomes, 2, [_value(r[1]) for r in rows],
                                              single_strand=single, threads=threads)
        for (m, v, i, o, snt), gi, go, gs in zip(rows, inm, outm, sent):
            assert (int(gi), int(go), int(gs)) == (_bases(i), _bases(o), int(snt)), (mode, v)
    # a vertex that is not in the graph has no edges
    inm, outm, sent = oracle.vertex_masks(genomes, 2, [_value("AT")], single_strand=single)
    assert (int(inm[0]), int(outm[0]), int(sent[0])) == (0, 0, 0)


# ------------------------------------------- two-pass == definition, tiny inputs

def _all_strings(maxlen):
    for n in range(1, maxlen + 1):
        for t in itertools.product(range(4), repeat=n):
            yield np.array(t, dtype=np.uint8)


@pytest.mark.parametrize("single", [False, True])
def test_twopass_equals_bruteforce_exhaustive(single):
    # every string of length <= 6, k = 1..4, a collision-heavy filter (pass 2
    # must clean up) and a roomy one
    for s in _all_strings(6):
        for k in range(1, min(4, s.size) + 1):
            want = oracle.bruteforce([s], k, single_strand=single)
            for b, h in ((32, 1), (2**12, 3)):
                tp = oracle.twopass([s], k, b, h, single_strand=single)
                assert list(tp.junctions[0]) == list(want[0]), (s, k, b, h)
                assert set(want[0]) <= set(tp.c1[0])


@pytest.mark.parametrize("single", [False, True])
def test_twopass_equals_bruteforce_random_multi(single):
    r = np.random.default_rng(7 if single else 8)
    for case in range(300):
        n = int(r.integers(1, 5))
        alphabet = int(r.integers(1, 5))
        gs = synth.random_genomes(1000 * int(single) + case, n, 0, 40, alphabet=alphabet,
                                  n_frac=float(r.choice([0.0, 0.1])))
        k = int(r.integers(1, 9))
        b = int(2 ** r.integers(5, 17))
        h = int(r.integers(1, 6))
        want = oracle.bruteforce(gs, k, single_strand=single)
        tp = oracle.twopass(gs, k, b, h, single_strand=single)
        assert as_sets(tp.junctions) == as_sets(want), (case, k, b, h)
        for c1, j in zip(tp.c1, want):
            assert set(j) <= set(c1)


def test_even_k_palindromes():
    # even k allows palindromic k-mers (own reverse complement)
    gs = [enc("ACGTACGTAATTGCGCAT"), enc("GGATCCAGCTTT"), enc("AATTAATTAATT")]
    for k in (2, 4, 6):
        want = oracle.bruteforce(gs, k)
        tp = oracle.twopass(gs, k, 2**12, 2)
        assert as_sets(tp.junctions) == as_sets(want)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("single", [False, True])
def test_homopolymer_every_position(single):
    # every k-mer of A^n is A^k, the first k-mer of the string: a sentinel
    for n, k in ((7, 3), (50, 25), (64, 63)):
        s = np.zeros(n, dtype=np.uint8)
        tp = oracle.twopass([s], k, 2**10, 3, single_strand=single)
        assert list(tp.junctions[0]) == list(range(n - k + 1))


def test_random_long_k_only_ends():
    # a random 20 kbp genome has no repeated 63-mer w.h.p.: only the two
    # sentinel positions are junctions
    s = synth.random_bases(synth.rng(99, 1), 20_000)
    k = 63
    tp = oracle.twopass([s], k, 2**20, 4)
    assert list(tp.junctions[0]) == [0, s.size - k]
    assert list(oracle.bruteforce([s], k)[0]) == [0, s.size - k]


def test_reverse_complement_mirror():
    # J(s-bar) = {|s|-k-i : i in J(s)}: junction status is a property of the
    # comprehensive graph, which s and s-bar generate alike
    gs = synth.random_genomes(5, 3, 200, 400, alphabet=3)
    k = 5
    fwd = oracle.twopass(gs, k, 2**14, 3).junctions
    rev = oracle.twopass([synth.reverse_complement(g) for g in gs], k, 2**14, 3).junctions
    for g, jf, jr in zip(gs, fwd, rev):
        assert sorted(g.size - k - int(i) for i in jf) == [int(x) for x in jr]


def test_duplicate_and_permuted_genomes():
    gs = synth.random_genomes(6, 3, 300, 500, alphabet=3)
    k = 6
    base = as_sets(oracle.twopass(gs, k, 2**14, 3).junctions)
    perm = as_sets(oracle.twopass(gs[::-1], k, 2**14, 3).junctions)[::-1]
    assert base == perm
    dup = as_sets(oracle.twopass(gs + [gs[0]], k, 2**14, 3).junctions)
    assert dup[:3] == base and dup[3] == base[0]


def test_n_runs_split_strings():
    # N splits a genome into separate strings: same junctions as the pieces
    a, b = enc("ACGGTACCATTG"), enc("TTGACCAGTAC")
    joined = np.concatenate([a, np.full(5, 4, np.uint8), b])
    k = 3
    j_joined = [int(x) for x in oracle.twopass([joined], k, 2**12, 3).junctions[0]]
    j_parts = oracle.twopass([a, b], k, 2**12, 3).junctions
    want = [int(x) for x in j_parts[0]] + [int(x) + a.size + 5 for x in j_parts[1]]
    assert j_joined == want


# ------------------------------------------------ invariants on a real workload

@pytest.fixture(scope="module")
def small_workload():
    gs = synth.plain_small(0)
    tp = oracle.twopass(gs, 25, 2**24, 3, with_distinct=True)
    return gs, tp


def test_plain_small_matches_bruteforce(small_workload):
    gs, tp = small_workload
    assert as_sets(oracle.bruteforce(gs, 25)) == as_sets(tp.junctions)


def test_candidates_superset_and_b_independence(small_workload):
    gs, tp = small_workload
    for c1, j in zip(tp.c1, tp.junctions):
        assert set(j.tolist()) <= set(c1.tolist())
    other = oracle.twopass(gs, 25, 2**18, 2)
    assert as_sets(other.junctions) == as_sets(tp.junctions)
    assert other.stats["marks_pass1"] > tp.stats["marks_pass1"]


def test_candidate_closure_under_normalised_kmer(small_workload):
    # a candidate set never splits the positions of one normalised k-mer
    gs, tp = small_workload
    for marks in (tp.c1, tp.junctions):
        marked, unmarked = set(), set()
        for g, m in zip(gs, marks):
            allpos = np.arange(g.size - 25 + 1, dtype=np.uint64)
            lo, hi, _ = oracle.vertices(g, 25, allpos)
            flag = np.zeros(allpos.size, bool)
            flag[m.astype(np.int64)] = True
            marked |= set(lo[flag].tolist())
            unmarked |= set(lo[~flag].tolist())
        assert not (marked & unmarked)


def test_edges_tile_each_string(small_workload):
    gs, tp = small_workload
    k = 25
    e = oracle.edges(gs, k, tp.junctions)
    for gi, g in enumerate(gs):
        mine = e[e[:, 0] == gi]
        # one string per genome (no N): edges chain from 0 to |s|-k
        assert mine.shape[0] == len(tp.junctions[gi]) - 1
        assert int((mine[:, 2] - mine[:, 1]).sum()) == g.size - k
        assert np.all(mine[1:, 1] == mine[:-1, 2])


def test_marks_decrease_per_pass(small_workload):
    # Table of marks per pass: pass 1 never adds marks, pass 2 never adds any
    _, tp = small_workload
    s = tp.stats
    assert s["positions"] >= s["marks_pass1"] >= s["marks_pass2"] > 0


# --------------------------------------- false-positive analysis (statistical)

def test_bloom_fill_and_false_positive_rate():
    # Theoretical Analysis section: a Bloom query for an absent element is a
    # false positive with q = (1 - e^{-hE/b})^h; a link is left marked with
    # p = 1 - (1 - q)^6; E[FP links] = L p.
    gs = synth.plain_small(1)
    k, b, h = 25, 2**20, 3
    tp = oracle.twopass(gs, k, b, h, with_distinct=True)
    E = tp.stats["distinct_edges"]
    rho = tp.stats["bloom_popcount"] / b
    rho_th = 1 - math.exp(-h * E / b)
    # fill: binomial-like spread over b bits
    assert abs(rho - rho_th) < 6 * math.sqrt(rho_th * (1 - rho_th) / b) + 1e-4

    # distinct links (normalised k-mers never junctions) and those left marked
    links, fp = set(), set()
    for g, c1, j in zip(gs, tp.c1, tp.junctions):
        allpos = np.arange(g.size - k + 1, dtype=np.uint64)
        lo, _, _ = oracle.vertices(g, k, allpos)
        isj = np.zeros(allpos.size, bool)
        isj[j.astype(np.int64)] = True
        isc = np.zeros(allpos.size, bool)
        isc[c1.astype(np.int64)] = True
        links |= set(lo[~isj].tolist())
        fp |= set(lo[isc & ~isj].tolist())
    L = len(links)
    q = (1 - math.exp(-h * E / b)) ** h
    p = 1 - (1 - q) ** 6
    mean, sd = L * p, math.sqrt(L * p * (1 - p))
    assert L > 10_000 and mean > 100
    assert abs(len(fp) - mean) < 6 * sd, (len(fp), mean, sd)


def test_roomy_filter_leaves_only_junctions():
    # with no filter collisions the first pass is already exact
    gs = synth.random_genomes(11, 3, 100, 300, alphabet=2)
    tp = oracle.twopass(gs, 7, 2**30, 4)
    assert as_sets(tp.c1) == as_sets(tp.junctions)


# ------------------------------------------------------ blocked filter variant

def _rc_codes(e):
    return np.array([3 - x for x in e[::-1]], dtype=np.uint8)


@pytest.mark.parametrize("k", [1, 2, 5, 24, 25, 31, 32, 40, 63])
def test_blocked_indices_structure(k):
    # all h bits of an edge share one 64-bit block; an edge and its reverse
    # complement get the same bits; for h <= 4 the distinct edges x.m.y around
    # one middle m (16, or 10 up to reverse complement when m is its own
    # reverse complement) use pairwise disjoint bits
    r = np.random.default_rng(100 + k)
    b = 2**16
    for _ in range(100):
        m = r.integers(0, 4, k - 1).astype(np.uint8)
        for h in (1, 3, 4, 7):
            sets = {}
            for x in range(4):
                for y in range(4):
                    e = np.concatenate([[x], m, [y]]).astype(np.uint8)
                    idx = oracle.blocked_indices(e, k, b, h)
                    assert len({i // 64 for i in idx}) == 1
                    assert idx == oracle.blocked_indices(_rc_codes(e), k, b, h)
                    assert all(0 <= i < b for i in idx)
                    key = min(tuple(e.tolist()), tuple(_rc_codes(e).tolist()))
                    sets[key] = set(idx)
            palindromic_middle = np.array_equal(m, _rc_codes(m))
            assert len(sets) == (10 if palindromic_middle else 16)
            if h <= 4:
                assert sum(len(v) for v in sets.values()) == len(set().union(*sets.values()))
                assert all(len(v) == h for v in sets.values())


@pytest.mark.parametrize("single", [False, True])
def test_blocked_twopass_equals_bruteforce(single):
    for s in _all_strings(5):
        for k in range(1, min(4, s.size) + 1):
            want = oracle.bruteforce([s], k, single_strand=single)
            for b, h in ((64, 1), (2**12, 3)):
                tp = oracle.twopass([s], k, b, h, single_strand=single, blocked=True)
                assert list(tp.junctions[0]) == list(want[0]), (s, k, b, h)
                assert set(want[0]) <= set(tp.c1[0])
    r = np.random.default_rng(17 if single else 18)
    for case in range(200):
        gs = synth.random_genomes(3000 + case, int(r.integers(1, 5)), 0, 60,
                                  alphabet=int(r.integers(1, 5)),
                                  n_frac=float(r.choice([0.0, 0.1])))
        k = int(r.integers(1, 12))
        b, h = int(2 ** r.integers(6, 16)), int(r.integers(1, 8))
        want = oracle.bruteforce(gs, k, single_strand=single)
        tp = oracle.twopass(gs, k, b, h, single_strand=single, blocked=True)
        assert as_sets(tp.junctions) == as_sets(want), (case, k, b, h)


def test_blocked_false_positive_rate():
    # Each link makes 3 queries in the block of its out-middle and 3 in the
    # block of its in-middle.  Model: a block holds n ~ Poisson(64E/b) edges of
    # other middles (edges of the queried middle use other bits), filling a
    # fraction f = 1 - (1 - 1/64)^(hn) of it; p = 1 - E[(1 - f^h)^3]^2.
    # Edges sharing a middle land in one block, so real block loads vary more
    # than Poisson and the measured rate sits 0-30% above the model.
    gs = synth.plain_small(1)
    k, b, h = 25, 2**20, 3
    tp = oracle.twopass(gs, k, b, h, with_distinct=True, blocked=True)
    E = tp.stats["distinct_edges"]
    lam = E * 64 / b
    keep = 0.0
    for n in range(200):
        pn = math.exp(-lam + n * math.log(lam) - math.lgamma(n + 1))
        f = 1 - (1 - 1 / 64) ** (h * n)
        keep += pn * (1 - f ** h) ** 3
    p = 1 - keep * keep
    links, fp = set(), set()
    for g, c1, j in zip(gs, tp.c1, tp.junctions):
        allpos = np.arange(g.size - k + 1, dtype=np.uint64)
        lo, _, _ = oracle.vertices(g, k, allpos)
        isj = np.zeros(allpos.size, bool)
        isj[j.astype(np.int64)] = True
        isc = np.zeros(allpos.size, bool)
        isc[c1.astype(np.int64)] = True
        links |= set(lo[~isj].tolist())
        fp |= set(lo[isc & ~isj].tolist())
    ratio = len(fp) / (len(links) * p)
    assert 0.95 < ratio < 1.3, ratio


def test_blocked_filter_has_no_false_negatives():
    gs = synth.plain_small(3)[:2]
    k, b, h = 25, 2**18, 4
    tp = oracle.twopass(gs, k, b, h, blocked=True)
    bits = np.unpackbits(tp.bloom.view(np.uint8), bitorder="little")
    r = np.random.default_rng(5)
    for g in gs:
        for j in r.integers(0, g.size - k - 1, 500):
            idx = oracle.blocked_indices(g[j:j + k + 1], k, b, h)
            assert all(bits[i] for i in idx)


# --------------------------------------------- Algorithm 3 (multiple rounds)

def _norm_value(codes, i, k, single=False):
    """Normalised value of the k-mer at i (first base most significant)."""
    fwd = 0
    rc = 0
    for t in range(k):
        fwd = fwd * 4 + int(codes[i + t])
        rc = rc * 4 + (3 - int(codes[i + k - 1 - t]))
    return fwd if single else min(fwd, rc)


@pytest.mark.parametrize("blocked", [False, True])
def test_rounds_one_is_algorithm_2(blocked):
    # the Multiple Rounds section: with l = 1, Algorithm 3 reduces to Algorithm 2
    gs = synth.random_genomes(31, 4, 200, 3000, alphabet=3, n_frac=0.01)
    for k, b, h in ((7, 2**12, 3), (25, 2**10, 2), (40, 2**14, 4)):
        r = oracle.rounds(gs, k, b, h, 1, blocked=blocked)
        t = oracle.twopass(gs, k, b, h, blocked=blocked)
        assert list(r.bounds) == [0, oracle.Q]
        assert np.array_equal(r.bloom, t.bloom)
        assert as_sets(r.c1) == as_sets(t.c1)
        assert as_sets(r.junctions) == as_sets(t.junctions)
        assert r.stats["marks_pass1"] == t.stats["marks_pass1"]


@pytest.mark.parametrize("single", [False, True])
def test_rounds_equal_bruteforce_random_multi(single):
    r = np.random.default_rng(41 if single else 42)
    for case in range(120):
        n = int(r.integers(1, 5))
        gs = synth.random_genomes(3000 + 500 * int(single) + case, n, 0, 60,
                                  alphabet=int(r.integers(1, 5)),
                                  n_frac=float(r.choice([0.0, 0.1])))
        k = int(r.integers(1, 9))
        b = int(2 ** r.integers(6, 14))
        h = int(r.integers(1, 5))
        l = int(r.choice([2, 3, 5, 16]))
        blocked = bool(case % 2)
        want = oracle.bruteforce(gs, k, single_strand=single)
        got = oracle.rounds(gs, k, b, h, l, single_strand=single, blocked=blocked)
        assert as_sets(got.junctions) == as_sets(want), (case, k, b, h, l, blocked)
        for c1, j in zip(got.c1, want):
            assert set(j) <= set(c1)


def test_partition_hand_examples():
    e = np.zeros(oracle.Q, dtype=np.uint64)
    e[:4] = 10
    # total 40: class 0 keeps subranges while their sum * l <= 40
    assert list(oracle.partition(e, 2)) == [0, 2, oracle.Q]
    assert list(oracle.partition(e, 3)) == [0, 1, 2, oracle.Q]
    assert list(oracle.partition(e, 4)) == [0, 1, 2, 3, oracle.Q]
    # uniform counters split evenly
    u = np.ones(oracle.Q, dtype=np.uint64)
    assert list(oracle.partition(u, 4)) == [0, 256, 512, 768, 1024]
    # a heavy subrange forms a class of its own, at least one subrange each
    h = np.ones(oracle.Q, dtype=np.uint64)
    h[0] = 100
    # total 1123, l = 2: 100 + 461 ones = 561 <= 561.5, one more would exceed
    assert list(oracle.partition(h, 2)) == [0, 462, oracle.Q]
    h[5] = 5000
    b = list(oracle.partition(h, 3))
    assert b[0] == 0 and b[-1] == oracle.Q and b == sorted(b)
    # the heavy subrange 5 ends class 0 (it cannot join: 5000 * 3 > total)
    assert b[1] == 5 and b[2] == 6
    # more classes than subranges with weight: trailing classes may be empty
    z = np.zeros(oracle.Q, dtype=np.uint64)
    z[0] = 1
    bz = list(oracle.partition(z, 3))
    assert bz[0] == 0 and bz[-1] == oracle.Q and bz == sorted(bz)


def test_partition_greedy_properties():
    r = np.random.default_rng(5)
    for _ in range(200):
        e = r.integers(0, 1000, oracle.Q).astype(np.uint64)
        e[r.random(oracle.Q) < 0.3] = 0
        l = int(r.integers(1, 40))
        b = [int(x) for x in oracle.partition(e, l)]
        total = int(e.sum())
        assert b[0] == 0 and b[-1] == oracle.Q and b == sorted(b) and len(b) == l + 1
        for c in range(l - 1):
            lo, hi = b[c], b[c + 1]
            s = int(e[lo:hi].sum())
            if hi - lo > 1:
                assert s * l <= total  # within the target
            if hi < oracle.Q and hi > lo:
                assert (s + int(e[hi])) * l > total  # as many subranges as fit


def test_census_hand_examples():
    # counters of the partition heuristic worked by hand (golden file)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "census_example.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for mode, text, k, counts in rows:
        k = int(k)
        want = np.zeros(oracle.Q, dtype=np.uint64)
        subs = set()
        for item in counts.split(","):
            kmer, c = item.split(":")
            sub = oracle.subrange(_value(kmer), k)
            subs.add(sub)
            want[sub] = int(c)
        assert len(subs) == len(counts.split(",")), "listed k-mers share a subrange"
        got = oracle.rounds([enc(text)], k, 2**12, 2, 2, single_strand=mode == "single")
        assert np.array_equal(got.counters, want), (mode, text)


def test_census_consistency_on_random_inputs():
    # consistency with the same counting rule over random inputs with N runs
    # (a check of the oracle's bookkeeping, not an independent pin: the hand
    # examples above are that)
    gs = synth.random_genomes(77, 3, 20, 300, alphabet=4, n_frac=0.02)
    for k, single in ((5, False), (12, True), (33, False)):
        want = np.zeros(oracle.Q, dtype=np.uint64)
        for g in gs:
            run = 0
            for j in range(g.size + 1):
                if j < g.size and g[j] < 4:
                    run += 1
                    continue
                start = j - run
                for i in range(start, j - k):
                    a = oracle.subrange(_norm_value(g, i, k, single), k)
                    z = oracle.subrange(_norm_value(g, i + 1, k, single), k)
                    want[a] += 1
                    if z != a:
                        want[z] += 1
                run = 0
        got = oracle.rounds(gs, k, 2**12, 2, 3, single_strand=single)
        assert np.array_equal(got.counters, want), k


def test_rounds_thin_the_candidates():
    # each round's filter holds only the edges next to its class, so a crowded
    # filter yields fewer false candidates with more rounds; J never changes
    gs = [g[:30000] for g in synth.plain_small(3)]
    base = oracle.twopass(gs, 25, 2**16, 2)
    prev = base.stats["marks_pass1"]
    for l in (2, 4, 8):
        r = oracle.rounds(gs, 25, 2**16, 2, l)
        assert as_sets(r.junctions) == as_sets(base.junctions)
        assert r.stats["marks_pass1"] < prev, l
        prev = r.stats["marks_pass1"]
        assert r.stats["bloom_popcount"] < base.stats["bloom_popcount"] * 1.0 * l


# ------------------------------------------------ long k (four-word values)

def _bigval(codes, i, k):
    v = 0
    for t in range(k):
        v = v * 4 + int(codes[i + t])
    return v


@pytest.mark.parametrize("k", [64, 65, 80, 100, 127])
def test_long_k_equals_bruteforce(k):
    r = np.random.default_rng(k)
    for case in range(12):
        gs = synth.random_genomes(9000 + 100 * k + case, int(r.integers(1, 4)), k - 5, 3 * k,
                                  alphabet=int(r.integers(1, 3)),
                                  n_frac=float(r.choice([0.0, 0.01])))
        for single in (False, True):
            want = oracle.bruteforce(gs, k, single_strand=single)
            for blocked in (False, True):
                tp = oracle.twopass(gs, k, 2**10, 2, single_strand=single, blocked=blocked)
                assert as_sets(tp.junctions) == as_sets(want), (k, case, single, blocked)
                ro = oracle.rounds(gs, k, 2**10, 2, 3, single_strand=single, blocked=blocked)
                assert as_sets(ro.junctions) == as_sets(want), (k, case, single, blocked)


def test_long_k_closed_forms():
    k = 100
    homo = np.zeros(400, np.uint8)
    tp = oracle.twopass([homo], k, 2**12, 3)
    assert list(tp.junctions[0]) == list(range(400 - k + 1))  # every k-mer is the sentinel
    g = synth.random_genomes(17, 1, 20000, 20000)[0]
    tp = oracle.twopass([g], k, 2**20, 3, blocked=True)
    assert list(tp.junctions[0]) == [0, g.size - k]
    # the reverse complement genome has the mirrored junctions
    rc = (3 - g[::-1]).astype(np.uint8)
    both = oracle.twopass([g, rc], k, 2**20, 3)
    assert [int(x) for x in both.junctions[1]] == [0, g.size - k]


def test_long_k_vertex_words():
    g = synth.random_genomes(23, 1, 500, 500)[0]
    for k in (64, 100, 127):
        pos = np.arange(0, g.size - k + 1, 37, dtype=np.uint64)
        words, strand = oracle.vertex_words(g, k, pos)
        for i, p in enumerate(pos):
            f = _bigval(g, int(p), k)
            r = _bigval((3 - g[int(p):int(p) + k][::-1]).astype(np.uint8), 0, k)
            m = min(f, r)
            assert [int(w) for w in words[i]] == [(m >> (64 * j)) & (M64 - 1) for j in range(4)]
            assert int(strand[i]) == (0 if f <= r else 1)


# --------------------------------------- sampled status and vertex masks

def _all_positions(gs, k):
    sg, sp = [], []
    for gi, g in enumerate(gs):
        run = 0
        for j in range(g.size + 1):
            if j < g.size and g[j] < 4:
                run += 1
                continue
            for i in range(j - run, j - k + 1):
                sg.append(gi)
                sp.append(i)
            run = 0
    return np.array(sg, dtype=np.uint32), np.array(sp, dtype=np.uint64)


@pytest.mark.parametrize("single", [False, True])
def test_sample_status_equals_bruteforce(single):
    # the junction status of every position by the streaming pass equals the
    # brute-force definition: N runs, even k (palindromes), k up to 127,
    # one and several threads, tiny alphabets (dense repeats)
    r = np.random.default_rng(31 + single)
    ks = list(range(1, 9)) + [12, 16, 25, 31, 32, 40, 63, 64, 100, 127]
    for case in range(90):
        k = ks[case % len(ks)]
        gs = synth.random_genomes(5000 + case, int(r.integers(1, 4)), max(1, k - 3), 3 * k + 40,
                                  alphabet=int(r.integers(1, 5)),
                                  n_frac=float(r.choice([0.0, 0.02, 0.1])))
        want = oracle.bruteforce(gs, k, single_strand=single)
        sg, sp = _all_positions(gs, k)
        threads = 1 + case % 3
        got = oracle.sample_status(gs, k, sg, sp, single_strand=single, threads=threads)
        want_status = np.zeros(sp.size, dtype=np.uint8)
        for i, (g, p) in enumerate(zip(sg, sp)):
            want_status[i] = int(p) in set(int(x) for x in want[int(g)])
        assert np.array_equal(got, want_status), (case, k, single)


def test_sample_status_packed_equals_codes():
    # the packed-input form (the library's input format) reads the same
    # strings: same status for samples drawn across strings and N runs
    r = np.random.default_rng(8)
    for case in range(12):
        k = int(r.choice([3, 11, 25, 33, 70]))
        gs = synth.random_genomes(6000 + case, 3, 200, 4000, alphabet=int(r.integers(2, 5)),
                                  n_frac=0.005)
        sg, sp = _all_positions(gs, k)
        pick = r.choice(sp.size, min(sp.size, 500), replace=False)
        packed = [synth.pack(g) + () for g in gs]
        packed = [(pk, g.size, runs) for (pk, runs), g in zip(packed, gs)]
        for single in (False, True):
            a = oracle.sample_status(gs, k, sg[pick], sp[pick], single_strand=single)
            b = oracle.sample_status(packed, k, sg[pick], sp[pick], single_strand=single,
                                     packed=True, threads=4)
            assert np.array_equal(a, b), (case, k, single)


def test_vertex_masks_long_strings_across_pieces():
    # strings longer than one work piece (4 Mbp) roll across piece borders:
    # a homopolymer's only vertex enters and leaves itself by its own base
    g = np.full(9_000_001, 2, dtype=np.uint8)   # G^n
    g[4_000_010] = 4                             # one N: two strings
    inm, outm, sent = oracle.vertex_masks([g], 25, [_value("G" * 25), _value("C" * 25)],
                                          threads=3)
    assert [int(x) for x in inm] == [1 << 2, 1 << 1]   # G^25 entered by G, C^25 by C
    assert [int(x) for x in outm] == [1 << 2, 1 << 1]
    assert [int(x) for x in sent] == [1, 1]
    # random genome: masks of sampled k-mers by the streaming pass equal a
    # direct scan of the 26-mers on both strands
    g = synth.random_genomes(4242, 1, 8_500_000, 8_500_000, alphabet=2)[0]
    k = 21
    pos = np.array([0, 3_999_980, 3_999_999, 4_000_000, 4_000_001, 8_499_979], dtype=np.uint64)
    vals = [_value("".join("ACGT"[c] for c in g[int(p):int(p) + k])) for p in pos]
    inm, outm, _ = oracle.vertex_masks([g], k, vals, threads=4)
    s = "".join("ACGT"[c] for c in g)
    rcs = s[::-1].translate(str.maketrans("ACGT", "TGCA"))
    for v, gi, go in zip(vals, inm, outm):
        text = "".join("ACGT"[(v >> (2 * (k - 1 - t))) & 3] for t in range(k))
        want_in = want_out = 0
        for src in (s, rcs):
            start = src.find(text)
            while start >= 0:
                if start > 0:
                    want_in |= 1 << "ACGT".index(src[start - 1])
                if start + k < len(src):
                    want_out |= 1 << "ACGT".index(src[start + k])
                start = src.find(text, start + 1)
        assert (int(gi), int(go)) == (want_in, want_out), text
