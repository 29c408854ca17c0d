"""Shared test helpers: run the GPU library and the CPU oracle on the same
seeded inputs and compare every output element by element."""
import numpy as np

import oracle
import paper_1602_05856_amd as tp
import synth


def to_genomes(codes_list):
    out = []
    for c in codes_list:
        packed, runs = synth.pack(c)
        out.append(tp.Genome(packed=packed, n_bases=int(np.asarray(c).size), n_runs=runs))
    return out


def gpu_run(codes_list, k, b, h, flags=0, plan=None, config=None):
    """Run the library's device path; returns (plan, result, bloom, c1 per genome)."""
    import torch
    if plan is None:
        plan = tp.Plan(to_genomes(codes_list), k, b, h, flags)
    if config:
        plan.config = config
    d_in = plan.upload()
    plan.run(d_in)
    res = plan.download()
    bloom = plan.debug_bloom()
    c1 = plan.bitmap_positions(plan.debug_candidates())
    torch.cuda.synchronize()
    return plan, res, bloom, c1


def oracle_run(codes_list, k, b, h, flags=0):
    single = bool(flags & tp.TP_FLAG_SINGLE_STRAND)
    o = oracle.twopass(codes_list, k, b, h, single_strand=single,
                       blocked=bool(flags & tp.TP_FLAG_BLOCKED_FILTER))
    junctions = o.c1 if flags & tp.TP_FLAG_PASS1_ONLY else o.junctions
    vx = [oracle.vertex_words(g, k, j, single_strand=single) for g, j in zip(codes_list, junctions)]
    edges = oracle.edges(codes_list, k, junctions)
    return o, junctions, vx, edges


def assert_parity(codes_list, k, b, h, flags=0, check_bloom=True, label="", config=None):
    plan, res, bloom, c1 = gpu_run(codes_list, k, b, h, flags, config=config)
    o, junctions, vx, edges = oracle_run(codes_list, k, b, h, flags)
    W = 1 if k <= 31 else (2 if k <= 63 else 4)
    where = "%s k=%d b=%d h=%d flags=%d" % (label, k, b, h, flags)
    if check_bloom:
        assert np.array_equal(bloom, o.bloom), "Bloom words differ " + where
    for g in range(len(codes_list)):
        assert np.array_equal(c1[g], o.c1[g]), "C1 differs, genome %d %s" % (g, where)
        got = res.junctions(g)
        assert np.array_equal(got, junctions[g]), "J differs, genome %d %s" % (g, where)
        words, strand = vx[g]
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        assert np.array_equal(res.vertex[a:z, :W], words[:, :W]), "vertex, genome %d %s" % (g, where)
        assert np.array_equal(res.strand[a:z], strand), "strand, genome %d %s" % (g, where)
    got_e = np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                      res.edges["to_pos"]], axis=1) if res.edges.size else np.zeros((0, 3), np.uint64)
    assert np.array_equal(got_e, edges.reshape(-1, 3)), "edges differ " + where
    st = res.stats
    assert st["candidates"] == o.stats["marks_pass1"], where
    assert st["junctions"] == sum(len(j) for j in junctions), where
    assert st["bloom_popcount"] == o.stats["bloom_popcount"], where
    assert st["positions"] == o.stats["positions"], where
    plan.close()
    return res, o
