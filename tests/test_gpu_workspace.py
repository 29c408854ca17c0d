"""GPU parity of the caller-memory entry points: tp_run_ws on torch-owned
workspace and output buffers (bit-exact against the oracle, on its own and
replayed from a captured HIP graph), its overflow reports, the exact-table
debug tap against the oracle's definition-based in/out edges of every
candidate k-mer, tp_build_batch and tp_server_poll."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_run, to_genomes

pytestmark = pytest.mark.gpu

SINGLE, PASS1, BLOCKED = 1, 2, 4
HERE = os.path.dirname(os.path.abspath(__file__))


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


def bits_to_positions(plan, words):
    return plan.bitmap_positions(words.cpu().numpy().view(np.uint64))


def ws_run(plan, d_in, kf=1.0, jf=1.0):
    """Lay out, allocate (torch), prepare and run; returns (ws, out) after a sync."""
    import torch
    plan.workspace_layout(kf, jf)
    ws, out = plan.alloc_workspace()
    plan.prepare_workspace(ws)
    plan.run_ws(d_in, ws, out)
    torch.cuda.synchronize()
    return ws, out


def check_ws_vs_oracle(codes, k, b, h, flags, rounds=1, label=""):
    import torch

    import paper_1602_05856_amd as tp
    plan = tp.Plan(to_genomes(codes), k, b, h, flags)
    plan.rounds = rounds
    d_in = plan.upload()
    ws, out = ws_run(plan, d_in)
    L = plan._ws_layout
    cnt = plan.ws_counts(out)
    where = "%s k=%d b=%d h=%d flags=%d rounds=%d" % (label, k, b, h, flags, rounds)
    assert cnt["status"] == 0, where
    res = plan.ws_result(out)
    single = bool(flags & SINGLE)
    if rounds == 1:
        o, junctions, vx, edges = oracle_run(codes, k, b, h, flags)
        c1_want, bloom_want = o.c1, o.bloom
    else:
        o = oracle.rounds(codes, k, b, h, rounds, single_strand=single,
                          blocked=bool(flags & BLOCKED))
        junctions = o.c1 if flags & PASS1 else o.junctions
        vx = [oracle.vertex_words(g, k, j, single_strand=single) for g, j in zip(codes, junctions)]
        edges = oracle.edges(codes, k, junctions)
        c1_want, bloom_want = o.c1, o.bloom
    W = L["kmer_words"]
    bloom = ws[L["ws_off_bloom"]:L["ws_off_bloom"] + b // 8].view(torch.int32)
    assert np.array_equal(bloom.cpu().numpy().view(np.uint32), bloom_want), "bloom " + where
    nw = plan.bitmap_words
    c1 = ws[L["ws_off_candidates"]:L["ws_off_candidates"] + 8 * nw].view(torch.int64)
    got_c1 = bits_to_positions(plan, c1)
    for g in range(len(codes)):
        assert np.array_equal(got_c1[g], c1_want[g]), "C1 genome %d %s" % (g, where)
        assert np.array_equal(res.junctions(g), junctions[g]), "J genome %d %s" % (g, where)
        words, strand = vx[g]
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        assert np.array_equal(res.vertex[a:z, :W], words[:, :W]), "vertex %d %s" % (g, where)
        assert np.array_equal(res.strand[a:z], strand), "strand %d %s" % (g, where)
    got_e = np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                      res.edges["to_pos"]], axis=1) if res.edges.size else np.zeros((0, 3),
                                                                                    np.uint64)
    assert np.array_equal(got_e, edges.reshape(-1, 3)), "edges " + where
    assert cnt["candidates"] == o.stats["marks_pass1"], where
    assert cnt["junctions"] == sum(len(j) for j in junctions), where
    assert cnt["positions"] == o.stats["positions"], where
    assert cnt["bloom_popcount"] == o.stats["bloom_popcount"], where
    plan.close()
    return cnt


@pytest.mark.parametrize("k", [5, 25, 29, 31, 40, 63, 100])
def test_ws_parity(k):
    gs = synth.random_genomes(300 + k, 3, 1000, 9000, alphabet=2, n_frac=0.001)
    gs += [synth.plain_small(2)[0][:20000]]
    for b, h, flags in ((2**16, 3, 0), (2**18, 4, BLOCKED), (2**12, 2, BLOCKED | SINGLE),
                        (2**16, 3, PASS1)):
        say("case: ws k=%d b=%d h=%d flags=%d" % (k, b, h, flags))
        check_ws_vs_oracle(gs, k, b, h, flags, label="ws")


@pytest.mark.parametrize("rounds", [2, 3, 8])
def test_ws_rounds_parity(rounds):
    gs = synth.random_genomes(41, 3, 2000, 8000, alphabet=3, n_frac=0.002)
    for k, flags in ((25, BLOCKED), (33, 0), (25, PASS1 | BLOCKED)):
        say("case: ws rounds=%d k=%d flags=%d" % (rounds, k, flags))
        check_ws_vs_oracle(gs, k, 2**14, 3, flags, rounds=rounds, label="ws-rounds")


def test_ws_edge_cases():
    k = 11
    A = synth.random_bases(synth.rng(77, 2), 5000)
    gs = [np.zeros(0, np.uint8), A[:k - 1], A[:k], A[:k + 1], np.full(50, 4, np.uint8),
          A[:2048], A[:2049], np.zeros(3000, np.uint8), A[:5000]]
    for flags in (0, BLOCKED, PASS1):
        say("case: ws edge lengths flags=%d" % flags)
        check_ws_vs_oracle(gs, k, 2**12, 2, flags, label="ws-edges")
    # nothing but genomes shorter than k: no positions, no kernels with work
    say("case: ws no positions")
    check_ws_vs_oracle([A[:5], np.zeros(0, np.uint8)], k, 2**10, 2, 0, label="ws-empty")


def test_ws_batch_parity():
    import paper_1602_05856_amd as tp
    import torch
    sets = [synth.random_genomes(900 + s, int(1 + s % 4), 0, 7000, alphabet=2 + s % 3,
                                 n_frac=0.002) for s in range(9)]
    k, h = 31, 4
    for flags in (BLOCKED, 0):
        bs = [2 ** (8 + s % 9) for s in range(len(sets))]
        plan = tp.Plan.batch([(to_genomes(c), b) for c, b in zip(sets, bs)], k, h, flags)
        d_in = plan.upload()
        say("case: ws batch of %d sets flags=%d" % (len(sets), flags))
        ws, out = ws_run(plan, d_in)
        cnt = plan.ws_counts(out)
        assert cnt["status"] == 0
        res = plan.ws_result(out)
        g = 0
        for s, codes in enumerate(sets):
            o, junctions, vx, edges = oracle_run(codes, k, bs[s], h, flags)
            for gi in range(len(codes)):
                assert np.array_equal(res.junctions(g + gi), junctions[gi]), (s, gi)
                words, strand = vx[gi]
                a, z = res.junction_offset[g + gi], res.junction_offset[g + gi + 1]
                assert np.array_equal(res.vertex[a:z, 0], words[:, 0]), (s, gi)
                assert np.array_equal(res.strand[a:z], strand), (s, gi)
            g += len(codes)
        # per-set counters in the workspace
        L = plan._ws_layout
        sc = ws[L["ws_off_set_counters"]:L["ws_off_set_counters"] + 64 * len(sets)].view(
            torch.int64).view(len(sets), 8).cpu().numpy().view(np.uint64)
        for s, codes in enumerate(sets):
            o = oracle.twopass(codes, k, bs[s], h, blocked=bool(flags & BLOCKED))
            assert int(sc[s, 0]) == o.stats["marks_pass1"], s
            assert int(sc[s, 2]) == o.stats["marks_pass2"], s
        plan.close()


def test_ws_full_size_digests():
    # the whole bacterial workload (62 x 5 Mbp, k = 25, b = 2^30, h = 4, blocked
    # filter) on caller memory, against the full oracle run's digests
    import paper_1602_05856_amd as tp
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from digests import digest_outputs
    rec = json.load(open(os.path.join(HERE, "golden", "bacterial_k25_blocked.json")))
    codes = synth.bacterial(0)
    plan = tp.Plan(to_genomes(codes), 25, 1 << 30, 4, BLOCKED)
    d_in = plan.upload()
    say("case: ws full-size bacterial k=25 blocked")
    ws, out = ws_run(plan, d_in, kf=0.2, jf=1.0)
    cnt = plan.ws_counts(out)
    assert cnt["status"] == 0, cnt
    res = plan.ws_result(out)
    L = plan._ws_layout
    import torch
    bloom = ws[L["ws_off_bloom"]:L["ws_off_bloom"] + (1 << 30) // 8].view(torch.int32)
    c1 = ws[L["ws_off_candidates"]:L["ws_off_candidates"] + 8 * plan.bitmap_words].view(
        torch.int64)
    ng = len(codes)
    junctions = [res.junctions(g) for g in range(ng)]
    vertex, strand = [], []
    for g in range(ng):
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        vertex.append(res.vertex[a:z, :1])
        strand.append(res.strand[a:z])
    edges = np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                      res.edges["to_pos"]], axis=1)
    got = digest_outputs(bloom.cpu().numpy().view(np.uint32), bits_to_positions(plan, c1),
                         junctions, vertex, strand, edges, 1)
    assert got["counts"] == rec["counts"]
    for key in ("bloom", "c1", "junctions", "vertex", "strand", "edges"):
        assert got[key] == rec[key], key
    plan.close()


def test_ws_graph_capture_replays():
    # a whole run captured as one graph and replayed: every replay equals the
    # eager run, with other eager work on the device between replays
    import paper_1602_05856_amd as tp
    import torch
    gs = synth.plain_small(0)
    for flags, rounds in ((BLOCKED, 1), (0, 3)):
        plan = tp.Plan(to_genomes(gs), 25, 2**24, 3, flags)
        plan.rounds = rounds
        d_in = plan.upload()
        ws, out = ws_run(plan, d_in, kf=0.5, jf=0.5)
        want = plan.ws_result(out)
        assert plan.ws_counts(out)["status"] == 0
        other = tp.Plan(to_genomes(gs[:2]), 31, 2**20, 2, BLOCKED)
        od = other.upload()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            plan.run_ws(d_in, ws, out, stream=s)  # warm up on the capture stream
            s.synchronize()
            with torch.cuda.graph(g, stream=s):
                plan.run_ws(d_in, ws, out, stream=s)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(4):
            say("case: ws graph replay %d flags=%d rounds=%d" % (rep, flags, rounds))
            out.fill_(0xA5)
            ws[:min(ws.numel(), 1 << 20)].fill_(0x5A)  # layout tables live here: prepare again
            plan.prepare_workspace(ws)
            g.replay()
            torch.cuda.synchronize()
            other.run(od)  # eager work of another plan in between
            torch.cuda.synchronize()
            got = plan.ws_result(out)
            assert plan.ws_counts(out)["status"] == 0
            assert np.array_equal(got.junction_offset, want.junction_offset)
            assert np.array_equal(got.junction_pos, want.junction_pos)
            assert np.array_equal(got.vertex, want.vertex)
            assert np.array_equal(got.strand, want.strand)
            assert np.array_equal(got.edges, want.edges)
        del g
        other.close()
        plan.close()


def test_ws_overflow_reports():
    import paper_1602_05856_amd as tp
    gs = synth.plain_small(1)
    plan = tp.Plan(to_genomes(gs), 25, 2**16, 3, 0)  # a crowded filter: many candidates
    d_in = plan.upload()
    full_ws, full_out = ws_run(plan, d_in)
    full = plan.ws_counts(full_out)
    assert full["status"] == 0
    want = plan.ws_result(full_out)
    # a table bound far below the distinct candidates: reported, no fault
    say("case: ws table overflow")
    ws, out = ws_run(plan, d_in, kf=1e-6, jf=1.0)
    assert plan._ws_layout["table_slots"] <= 1024 + 4096
    assert plan.ws_counts(out)["status"] & tp.TP_WS_TABLE_OVERFLOW
    # an output bound below the junctions: reported, junction offsets true,
    # the junctions that fit are the first ones
    say("case: ws output overflow")
    ws, out = ws_run(plan, d_in, kf=1.0, jf=0.01)
    c = plan.ws_counts(out)
    assert c["status"] == tp.TP_WS_OUTPUT_OVERFLOW
    assert c["junctions"] == full["junctions"]
    mj = plan._ws_layout["max_junctions"]
    assert mj < full["junctions"]
    v = plan.ws_views(out)
    assert np.array_equal(v["joff"].cpu().numpy().view(np.uint64), want.junction_offset)
    assert np.array_equal(v["pos"][:mj].cpu().numpy().view(np.uint64), want.junction_pos[:mj])
    plan.close()


# ---------------------------------------------------------- table debug tap

def check_table_tap(k, config=None):
    # every candidate k-mer's in/out edge mask in the exact table equals the
    # oracle's in/out edges of that vertex in the comprehensive graph
    import paper_1602_05856_amd as tp
    gs = synth.random_genomes(700 + k, 3, 500, 5000, alphabet=2, n_frac=0.002)
    for flags in (0, BLOCKED, SINGLE):
        single = bool(flags & SINGLE)
        plan = tp.Plan(to_genomes(gs), k, 2**13, 3, flags)
        if config:
            plan.config = config
        d_in = plan.upload()
        plan.run(d_in)
        keys, masks = plan.debug_table()
        W = keys.shape[1]
        got = {}
        for row, m in zip(keys, masks):
            v = sum(int(row[i]) << (64 * i) for i in range(W))
            assert v not in got, "a k-mer holds two slots"
            got[v] = int(m)
        o = oracle.twopass(gs, k, 2**13, 3, single_strand=single, blocked=bool(flags & BLOCKED))
        cand = set()
        for g, c1 in zip(gs, o.c1):
            words, _ = oracle.vertex_words(g, k, c1, single_strand=single)
            for wrow in words:
                cand.add(sum(int(wrow[i]) << (64 * i) for i in range(4)))
        say("case: table tap k=%d flags=%d: %d keys, %d candidate k-mers" % (
            k, flags, len(got), len(cand)))
        assert set(got) == cand, "table keys differ from the candidate k-mers"
        vals = sorted(cand)
        inm, outm, _ = oracle.vertex_masks(gs, k, vals, single_strand=single)
        for v, i, o_ in zip(vals, inm, outm):
            assert got[v] == int(i) | int(o_) << 4, (k, flags, v)
        assert plan.stats()["table_keys"] == len(cand)
        if config and config.get("record_binned") == 2:
            assert plan.stats()["record_passes"] >= 1
        plan.close()


@pytest.mark.parametrize("k", [5, 25, 29, 40, 63, 100, 127])
def test_table_tap_matches_oracle_edges(k):
    check_table_tap(k)


@pytest.mark.parametrize("k", [5, 25])
def test_table_tap_of_binned_record(k):
    # the table the binned record builds (blocks in LDS, several passes)
    check_table_tap(k, {"record_binned": 2, "table_shape": 2, "record_passes": 2})


# ------------------------------------------------- batch build, server poll

def test_build_batch_equals_each_set_alone():
    import paper_1602_05856_amd as tp
    sets = [synth.random_genomes(1300 + s, 1 + s % 3, 100, 6000, alphabet=3, n_frac=0.003)
            for s in range(6)]
    k, h = 25, 3
    for flags in (0, BLOCKED):
        bs = [2 ** (10 + s) for s in range(len(sets))]
        say("case: build_batch flags=%d" % flags)
        results = tp.build_batch([(to_genomes(c), b) for c, b in zip(sets, bs)], k, h, flags)
        assert len(results) == len(sets)
        for s, (codes, res) in enumerate(zip(sets, results)):
            o, junctions, vx, edges = oracle_run(codes, k, bs[s], h, flags)
            for g in range(len(codes)):
                assert np.array_equal(res.junctions(g), junctions[g]), (s, g)
            got_e = np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                              res.edges["to_pos"]], axis=1) if res.edges.size else \
                np.zeros((0, 3), np.uint64)
            assert np.array_equal(got_e, edges.reshape(-1, 3)), s
            assert res.stats["candidates"] == o.stats["marks_pass1"], s


def test_server_poll():
    import time

    import paper_1602_05856_amd as tp
    jobs = [synth.random_genomes(1500 + j, 2, 1000, 30000, alphabet=3) for j in range(8)]
    srv = tp.Server(hbm_budget=8 << 30, workers=2, max_batch=4)
    ids = [srv.submit(to_genomes(c), 25, 2**18, 3, BLOCKED) for c in jobs]
    pending = dict(zip(ids, jobs))
    t0 = time.time()
    say("case: server poll, %d jobs" % len(ids))
    while pending and time.time() - t0 < 60:
        for jid in list(pending):
            got = srv.poll(jid)
            if got is None:
                continue
            res, info = got
            codes = pending.pop(jid)
            o = oracle.twopass(codes, 25, 2**18, 3, blocked=True)
            for g in range(len(codes)):
                assert np.array_equal(res.junctions(g), o.junctions[g]), (jid, g)
            with pytest.raises(tp.TwoPaCoError):
                srv.poll(jid)  # forgotten once handed out
        time.sleep(0.005)
    assert not pending, "jobs did not finish"
    srv.close()
