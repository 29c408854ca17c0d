"""Serving loop: jobs submitted together are batched and overlapped, and
each job's result is bit-identical to a build of that job alone (tolerance
0).  Admission by HBM budget, failure of a job too large for the budget, and
buffer reuse by a warm server are checked too."""
import sys

import numpy as np
import pytest

import synth
from helpers import oracle_run, to_genomes

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


def job_mix(seed, n_small=10, n_medium=3, n_large=1):
    """(codes, k, b, h, flags) per job: small k=25 sets, medium k=31 sets and
    a k=63 set, sizes scaled down from the serving workload's classes."""
    import paper_1602_05856_amd as tp
    r = np.random.default_rng(seed)
    jobs = []
    for cls, n, lo, hi, k in (("small", n_small, 50e3, 400e3, 25),
                              ("medium", n_medium, 1e6, 3e6, 31),
                              ("large", n_large, 4e6, 6e6, 63)):
        for i in range(n):
            total = float(np.exp(r.uniform(np.log(lo), np.log(hi))))
            g = int(r.integers(2, 6))
            codes = synth.genome_set(synth.rng(77, seed, len(jobs)), int(total / g), g)
            b = tp.bloom_bits_for(to_genomes(codes), k)
            flags = BLOCKED if i % 3 else 0
            jobs.append((codes, k, b, 4, flags))
    return jobs


def alone(codes, k, b, h, flags):
    import paper_1602_05856_amd as tp
    plan = tp.Plan(to_genomes(codes), k, b, h, flags)
    d_in = plan.upload()
    plan.run(d_in)
    res = plan.download()
    plan.close()
    return res


def assert_same(a, b, where):
    for f in ("junction_offset", "junction_pos", "vertex", "strand"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), "%s %s" % (where, f)
    assert np.array_equal(a.edges, b.edges), where + " edges"
    for f in ("positions", "candidates", "junctions", "edges", "bloom_popcount"):
        assert a.stats[f] == b.stats[f], "%s %s" % (where, f)


def test_alone_vs_mix_bit_exact():
    import paper_1602_05856_amd as tp
    jobs = job_mix(1)
    say("case: serving mix of %d jobs" % len(jobs))
    srv = tp.Server(hbm_budget=64 << 30, workers=3, max_batch=8,
                    batch_max_bases=2_000_000, batch_total_bases=50_000_000)
    packed = [to_genomes(c) for c, _, _, _, _ in jobs]  # submit in a tight loop
    ids = [srv.submit(g, k, b, h, f) for g, (_, k, b, h, f) in zip(packed, jobs)]
    got = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert max(info["batch_jobs"] for _, info in got) > 1, "no job was batched"
    for n, ((codes, k, b, h, f), (res, info)) in enumerate(zip(jobs, got)):
        assert info["end_s"] >= info["start_s"] >= info["submit_s"]
        assert_same(res, alone(codes, k, b, h, f), "job %d (k=%d, batch of %d)" %
                    (n, k, info["batch_jobs"]))
    # two small jobs straight against the oracle as well
    for n in (0, 1):
        codes, k, b, h, f = jobs[n]
        o, junctions, vx, edges = oracle_run(codes, k, b, h, f)
        res = got[n][0]
        for g in range(len(codes)):
            assert np.array_equal(res.junctions(g), junctions[g])
        assert res.stats["candidates"] == o.stats["marks_pass1"]


def test_budget_admission_and_oversized_job():
    import paper_1602_05856_amd as tp
    jobs = job_mix(2, n_small=4, n_medium=2, n_large=0)
    say("case: serving under a tight budget")
    # enough for about one medium job at a time
    srv = tp.Server(hbm_budget=600 << 20, workers=2, max_batch=4,
                    batch_max_bases=1_000_000, batch_total_bases=4_000_000)
    ids = [srv.submit(to_genomes(c), k, b, h, f) for c, k, b, h, f in jobs]
    huge = [np.zeros(300_000_000, np.uint8)]
    big_id = srv.submit(to_genomes(huge), 25, 1 << 30, 4, 0)
    got = [srv.wait(i) for i in ids]
    with pytest.raises(tp.TwoPaCoError) as e:
        srv.wait(big_id)
    assert e.value.status == tp.TP_ENOMEM
    st = srv.stats()
    srv.close()
    assert st["failed"] == 1
    assert st["peak_held_bytes"] <= 600 << 20, st
    for (codes, k, b, h, f), (res, info) in zip(jobs, got):
        assert_same(res, alone(codes, k, b, h, f), "budgeted job k=%d" % k)


def test_table_budget_splits_large_jobs_into_rounds():
    """A server-wide cap on any job's exact tables: a job whose one-round
    table would exceed it is built in rounds (Algorithm 3), with the
    junctions, vertices, strands and edges of its one-round build (the
    candidate count differs: each round's filter holds fewer edges)."""
    import paper_1602_05856_amd as tp
    codes, k, b, h, f = job_mix(9, n_small=0, n_medium=0, n_large=1)[0]
    one = alone(codes, k, b, h, f)
    assert one.stats["rounds"] == 1
    table_mib = one.stats["table_capacity"] * 17 / 2**20  # two key words and a mask byte
    cap = max(1, int(table_mib / 4))
    say("case: serving with a %d MiB table cap (one-round table %.1f MiB)" % (cap, table_mib))
    srv = tp.Server(hbm_budget=8 << 30, workers=1, max_batch=1, table_budget_mib=cap)
    res, info = srv.wait(srv.submit(to_genomes(codes), k, b, h, f))
    srv.close()
    assert res.stats["rounds"] > 1, res.stats["rounds"]
    for fld in ("junction_offset", "junction_pos", "vertex", "strand"):
        assert np.array_equal(getattr(res, fld), getattr(one, fld)), fld
    assert np.array_equal(res.edges, one.edges)
    assert res.stats["junctions"] == one.stats["junctions"]


def test_warm_server_reuses_buffers():
    import paper_1602_05856_amd as tp
    jobs = job_mix(3, n_small=3, n_medium=1, n_large=0)
    say("case: warm server buffer reuse")
    srv = tp.Server(hbm_budget=32 << 30, workers=1, max_batch=1)
    for c, k, b, h, f in jobs:
        srv.wait(srv.submit(to_genomes(c), k, b, h, f))
    held = srv.stats()["held_bytes"]
    assert held > 0
    for c, k, b, h, f in jobs:
        srv.wait(srv.submit(to_genomes(c), k, b, h, f))
    st = srv.stats()
    srv.close()
    assert st["held_bytes"] == held and st["peak_held_bytes"] == held


def test_express_workers_take_small_jobs_only():
    """With one express worker on CUs of its own, no job above batch_max_bases
    runs on it, every job of at most batch_max_bases runs on it (the CU split
    gives small jobs to the express lane only), and every job still equals
    its build alone."""
    import paper_1602_05856_amd as tp
    jobs = job_mix(4, n_small=8, n_medium=3, n_large=2)
    say("case: serving with an express worker, %d jobs" % len(jobs))
    limit = 500_000
    srv = tp.Server(hbm_budget=64 << 30, workers=3, max_batch=4, batch_max_bases=limit,
                    batch_total_bases=2_000_000, express_workers=1, express_cus=32)
    packed = [to_genomes(c) for c, _, _, _, _ in jobs]
    # large jobs first, so the general workers are busy when the small ones arrive
    order = sorted(range(len(jobs)), key=lambda n: -sum(int(c.size) for c in jobs[n][0]))
    ids = {n: srv.submit(packed[n], *jobs[n][1:]) for n in order}
    got = {n: srv.wait(ids[n]) for n in order}
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs) and st["failed"] == 0
    express = 2  # workers 0..2, the last is the express one
    ran_express = 0
    for n, (codes, k, b, h, f) in enumerate(jobs):
        res, info = got[n]
        if info["bases"] > limit:
            assert info["worker"] != express, "job %d (%d bases) ran on the express worker" % (
                n, info["bases"])
        else:
            assert info["worker"] == express, "small job %d ran on worker %d" % (
                n, info["worker"])
        ran_express += info["worker"] == express
        assert_same(res, alone(codes, k, b, h, f), "job %d" % n)
    assert ran_express > 0, "the express worker ran nothing"


def packed_set(codes):
    out = []
    for c in codes:
        pk, runs = synth.pack(c)
        out.append((pk, int(c.size), runs))
    return out


@pytest.mark.timeout(1200)
def test_serving_pool_full_size():
    """The serving workload's pool at full size (8 sets of 1-5 Mbp at k = 25,
    3 of 50-200 Mbp at k = 31, 3 of 1-3 Gbp at k = 63; blocked filter at 16
    bits per (k+1)-mer, h = 4), all submitted at once to a server configured
    as bench.py configures it: every small and medium job's junctions,
    vertices, strands and edges against the digests of the oracle run on
    that set (tests/golden/serving_pool.json, oracle only), and every large
    job's junction status at 20,000 uniformly sampled positions against the
    oracle's definition-based pass."""
    import json
    import os
    import time

    import oracle
    import paper_1602_05856_amd as tp
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    from digests import digest_outputs
    path = os.path.join(here, "golden", "serving_pool.json")
    rec = {(r["class"], r["index"]): r for r in json.load(open(path))["sets"]}
    entries = synth.serving_entries(0)
    srv = tp.Server(hbm_budget=200 << 30, workers=3, max_batch=32,
                    batch_max_bases=20_000_000, batch_total_bases=400_000_000, wg_per_cu=4,
                    express_workers=1)
    jobs = []
    t0 = time.time()
    for e in entries:
        name, k, i, glen, g = e
        codes = synth.serving_set(0, e)
        pk = packed_set(codes)
        del codes
        gs = [tp.Genome(packed=p, n_bases=n, n_runs=r) for p, n, r in pk]
        b = tp.bloom_bits_for(gs, k)
        if (name, i) in rec:
            assert b == rec[(name, i)]["bloom_bits"], (name, i)
        jobs.append((e, pk, b, srv.submit(gs, k, b, 4, BLOCKED)))
        say("submitted %s %d: %.1f Mbp (%.0f s)" % (name, i, glen * g / 1e6, time.time() - t0))
    results = []
    for e, pk, b, jid in jobs:
        res, info = srv.wait(jid)
        results.append((e, pk, res))
        say("done %s %d: %d junctions, run %.0f ms" % (e[0], e[2], res.stats["junctions"],
                                                        info["run_ms"]))
    st = srv.stats()
    srv.close()
    assert st["failed"] == 0
    for (name, k, i, glen, g), pk, res in results:
        W = 1 if k <= 31 else 2
        if (name, i) in rec:
            want = rec[(name, i)]
            ng = len(pk)
            off = res.junction_offset
            got = digest_outputs(np.zeros(1, np.uint32), [[]] * ng,
                                 [res.junctions(x) for x in range(ng)],
                                 [res.vertex[off[x]:off[x + 1], :W] for x in range(ng)],
                                 [res.strand[off[x]:off[x + 1]] for x in range(ng)],
                                 np.stack([res.edges["genome"].astype(np.uint64),
                                           res.edges["from_pos"], res.edges["to_pos"]], axis=1),
                                 W)
            for key in ("junctions", "vertex", "strand", "edges"):
                assert got[key] == want[key], (name, i, key)
            assert res.stats["junctions"] == want["counts"]["junctions"]
            continue
        # large: sampled junction status against the oracle's definition
        r = np.random.default_rng(100 + i)
        lens = np.array([max(0, n - k + 1) for _, n, _ in pk], dtype=np.int64)
        sg = r.choice(len(pk), 20000, p=lens / lens.sum()).astype(np.uint32)
        sp = np.array([r.integers(0, lens[x]) for x in sg], dtype=np.uint64)
        t1 = time.time()
        want = oracle.sample_status(pk, k, sg, sp, packed=True)
        got = np.zeros(sp.size, dtype=np.uint8)
        for x in range(len(pk)):
            sel = np.flatnonzero(sg == x)
            J = res.junctions(x)
            at = np.searchsorted(J, sp[sel])
            hit = at < J.size
            hit[hit] = J[at[hit]] == sp[sel][hit]
            got[sel] = hit
        say("large %d: %d of 20000 sampled positions are junctions (oracle %.0f s)" % (
            i, int(want.sum()), time.time() - t1))
        assert np.array_equal(got, want), (name, i, int((got != want).sum()))
