"""The primate-scale workload (8 genomes of 3 Gbp from one base, 1-8%
pairwise divergence, interspersed repeats, N runs; k=25, b=2^36, h=5).

At 1/1000 scale every output is checked against the oracle.  At full scale
(24 Gbp) the two-pass oracle cannot run, so 200,000 positions drawn uniformly
from all k-mer positions are checked against the oracle's definition-based
streaming pass (junction status of each sampled k-mer from its in- and
out-edges in the comprehensive graph), and the rest against properties that
hold at any size: the junctions do not depend on the filter or the rounds (a
blocked filter in one round gives the same bitmap), junctions are candidates,
every string's first and last k-mer is a junction, sampled vertices and
strands are the normalised k-mers of the genome (recomputed on the host), and
sampled edges join consecutive junctions of one genome."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from helpers import assert_parity

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


@pytest.mark.parametrize("flags", [0, BLOCKED])
def test_primate_reduced_scale_parity(flags):
    codes = synth.primate(0, 0.001)  # 8 x 3 Mbp, same recipe
    say("case: primate 1/1000 scale flags=%d, %.1f Mbp" % (flags, sum(c.size for c in codes) / 1e6))
    assert_parity(codes, 25, 2**26, 5, flags=flags, label="primate-0.001")


class DevArray:
    """__cuda_array_interface__ over device memory the plan owns."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3}


def dev_view(ptr, n, typestr):
    import torch
    return torch.as_tensor(DevArray(ptr, n, typestr), device="cuda")


def popcount_bytes(t):
    import torch
    table = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64,
                         device=t.device)
    b = t.view(torch.uint8)
    chunk = 1 << 27
    return sum(int(table[b[i:i + chunk].long()].sum()) for i in range(0, b.numel(), chunk))


def sample_positions(gs, k, n, seed):
    """n k-mer positions drawn uniformly from all positions of all strings:
    (genome, position) arrays, sorted."""
    starts, counts, owner = [], [], []
    for g, (_, m, runs) in enumerate(gs):
        cuts = [0]
        for s, ln in runs:
            cuts += [int(s), int(s + ln)]
        cuts.append(m)
        for a, z in np.array(cuts, dtype=np.int64).reshape(-1, 2):
            if z - a >= k:
                starts.append(a)
                counts.append(z - a - k + 1)
                owner.append(g)
    cum = np.concatenate([[0], np.cumsum(counts)])
    r = np.random.default_rng(seed)
    idx = np.sort(r.choice(int(cum[-1]), n, replace=False))
    which = np.searchsorted(cum, idx, side="right") - 1
    pos = np.array(starts, dtype=np.int64)[which] + (idx - cum[which])
    return np.array(owner, dtype=np.uint32)[which], pos.astype(np.uint64)


@pytest.mark.timeout(1500)
def test_primate_full_size_invariants():
    import torch

    import paper_1602_05856_amd as tp
    k = 25
    gs = synth.primate(0, 1.0, packed=True)
    say("case: primate full size, %.2f Gbp generated" % (sum(m for _, m, _ in gs) / 1e9))
    genomes = [tp.Genome(packed=p, n_bases=m, n_runs=r) for p, m, r in gs]

    # run A: the configured standard filter (two rounds keep the table small)
    plan = tp.Plan(genomes, k, 1 << 36, 5, 0)
    d_in = plan.upload()
    plan.rounds = 2
    plan.run(d_in)
    st = plan.stats()
    say("run A: %d candidates, %d junctions, %d edges, %.1f ms" % (
        st["candidates"], st["junctions"], st["edges"], st["ms_total"]))
    nw = plan.bitmap_words
    out = plan.device_outputs()
    J = dev_view(out["junction_bits"], nw, "<i8").clone()
    C1 = dev_view(out["candidates"], nw, "<i8").clone()
    assert not bool(torch.bitwise_and(J, torch.bitwise_not(C1)).any()), "a junction is no candidate"
    assert popcount_bytes(J) == st["junctions"]
    assert popcount_bytes(C1) == st["candidates"]
    gbase = [plan.genome_offset(g) * 4 for g in range(len(genomes))]
    nj = out["n_junctions"]
    assert nj == st["junctions"] and out["n_edges"] == st["edges"]
    joff = dev_view(out["junction_offset"], len(genomes) + 1, "<i8").cpu().numpy()

    # every string's first and last k-mer is a junction
    Jh = J.cpu().numpy().view(np.uint64)

    def bit(gp):
        gp = np.asarray(gp, dtype=np.uint64)
        return (Jh[gp >> np.uint64(6)] >> (gp & np.uint64(63))) & np.uint64(1)

    # sampled junction status against the oracle's definition-based pass
    sg, sp = sample_positions(gs, k, 200_000, seed=11)
    t0 = time.time()
    want = oracle.sample_status(gs, k, sg, sp, packed=True)
    say("oracle status of %d sampled positions in %.0f s: %d junctions" % (
        sp.size, time.time() - t0, int(want.sum())))
    got = bit(np.array(gbase, dtype=np.uint64)[sg.astype(np.int64)] + sp).astype(np.uint8)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%d sampled positions differ, first genome %d position %d" % (
        bad.size, int(sg[bad[0]]), int(sp[bad[0]]))
    assert 0 < int(want.sum()) < sp.size

    for g, (_, m, runs) in enumerate(gs):
        cuts = [0]
        for s, ln in runs:
            cuts += [int(s), int(s + ln)]
        cuts.append(m)
        ends = np.array(cuts, dtype=np.int64).reshape(-1, 2)
        ends = ends[ends[:, 1] - ends[:, 0] >= k]
        assert bit(gbase[g] + ends[:, 0]).all(), "genome %d: a string start is no junction" % g
        assert bit(gbase[g] + ends[:, 1] - k).all(), "genome %d: a string end is no junction" % g

    # sampled junctions: vertex and strand are the normalised k-mer at the position
    r = np.random.default_rng(1)
    idx = np.sort(r.choice(nj, 20000, replace=False)).astype(np.int64)
    it = torch.from_numpy(idx).cuda()
    pos = dev_view(out["junction_pos"], nj, "<i8")[it].cpu().numpy().astype(np.uint64)
    vx = dev_view(out["vertex"], nj, "<i8")[it].cpu().numpy().view(np.uint64)
    sd = dev_view(out["strand"], nj, "|u1")[it].cpu().numpy()
    gen = np.searchsorted(joff, idx, side="right") - 1
    kmers = []
    for g, p in zip(gen, pos):
        packed = gs[g][0]
        j = np.arange(int(p), int(p) + k)
        kmers.append((packed[j >> 2] >> (2 * (j & 3)).astype(np.uint8)) & 3)
    flat = np.concatenate(kmers).astype(np.uint8)
    want_w, want_s = oracle.vertex_words(flat, k, np.arange(0, flat.size, k, dtype=np.uint64))
    assert np.array_equal(vx, want_w[:, 0]), "sampled vertex ids differ"
    assert np.array_equal(sd, want_s), "sampled strands differ"
    assert bit(np.array([gbase[g] for g in gen], dtype=np.uint64) + pos).all()

    # sampled edges join consecutive junctions of one genome
    ne = out["n_edges"]
    eidx = torch.from_numpy(np.sort(r.choice(ne, 20000, replace=False)).astype(np.int64)).cuda()
    ew = dev_view(out["edges"], ne * 3, "<i8").view(-1, 3)[eidx].cpu().numpy().view(np.uint64)
    eg, ef, et = ew[:, 0] & np.uint64(0xFFFFFFFF), ew[:, 1], ew[:, 2]
    assert (ef < et).all() and (eg < len(genomes)).all()
    base = np.array(gbase, dtype=np.uint64)[eg.astype(np.int64)]
    assert bit(base + ef).all() and bit(base + et).all()
    for b0, f, t in zip(base, ef, et):
        if t - f <= 4096:
            between = b0 + np.arange(int(f) + 1, int(t), dtype=np.uint64)
            assert not bit(between).any(), "an edge skips a junction"
    plan.close()
    del C1

    # run B: a blocked filter gives the same junctions, in one round.  With a
    # power-of-two table (2^34 slots) the table and the outputs do not fit HBM
    # together: the first run frees the table before compaction, the second
    # frees the first run's outputs before the table.  The third run takes the
    # default sizing (an any-size table of ~1.1e10 slots that fits).
    plan = tp.Plan(genomes, k, 1 << 36, 5, BLOCKED)
    plan.rounds = 1
    for rep, shape in ((0, 1), (1, 1), (2, 0)):
        plan.config = {"table_shape": shape}
        plan.run(d_in)
        st2 = plan.stats()
        say("run B%d (blocked, one round, table_shape %d): %d candidates, %d junctions, "
            "%d table slots, %.1f ms" % (rep, shape, st2["candidates"], st2["junctions"],
                                         st2["table_capacity"], st2["ms_total"]))
        home = st2["table_capacity"] - 4096
        assert (home & (home - 1) == 0) == (shape == 1), home
        J2 = dev_view(plan.device_outputs()["junction_bits"], nw, "<i8")
        assert torch.equal(J, J2), "junctions depend on the filter or the rounds"
        assert st2["edges"] == st["edges"]
    plan.close()
