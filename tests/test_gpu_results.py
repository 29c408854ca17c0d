"""Host results view the library's page-locked result block (no copy): the
arrays stay valid after the plan is closed and while other results come and
go, slices outlive their Result, and a block reused from the library's cache
holds the new result."""
import gc
import sys

import numpy as np
import pytest

import synth
from helpers import oracle_run, to_genomes

pytestmark = pytest.mark.gpu


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


def test_result_views_outlive_plan_and_churn():
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(500, 3, 20_000, 60_000, alphabet=3, n_frac=0.001)
    k = 25
    _, junctions, vx, _ = oracle_run(codes, k, 2**18, 3)
    say("case: result lifetime, 3 genomes, k=25")
    plan = tp.Plan(to_genomes(codes), k, 2**18, 3)
    d_in = plan.upload()
    plan.run(d_in)
    res = plan.download()
    first = res.junctions(0)                # a slice of the block
    vertex = res.vertex
    plan.close()
    del d_in
    # other results are allocated and freed meanwhile (they may reuse cached blocks)
    for seed in range(3):
        other = tp.twopaco_build(to_genomes(synth.random_genomes(600 + seed, 2, 5000, 20_000)),
                                 k, 2**16, 3)
        assert other.stats["junctions"] > 0
        del other
        gc.collect()
    for g in range(len(codes)):
        assert np.array_equal(res.junctions(g), junctions[g])
    del res
    gc.collect()
    assert np.array_equal(first, junctions[0])   # the slice keeps the block alive
    assert np.array_equal(vertex[:len(first), 0], vx[0][0][:, 0])
    del first, vertex
    gc.collect()


def test_repeated_downloads_match():
    import paper_1602_05856_amd as tp
    codes = synth.random_genomes(700, 4, 10_000, 40_000, alphabet=2)
    plan = tp.Plan(to_genomes(codes), 21, 2**18, 4, tp.TP_FLAG_BLOCKED_FILTER)
    d_in = plan.upload()
    plan.run(d_in)
    say("case: repeated downloads, 4 genomes, k=21")
    ref = plan.download()
    keep = [np.array(a) for a in (ref.junction_pos, ref.vertex, ref.strand, ref.edges)]
    for rep in range(4):
        del ref
        gc.collect()                 # the block goes back to the cache
        ref = plan.download()        # and may be handed out again here
        got = (ref.junction_pos, ref.vertex, ref.strand, ref.edges)
        for a, b in zip(keep, got):
            assert np.array_equal(a, b), rep
    plan.close()
