"""Full-size parity on the bacterial workload (62 x 5 Mbp, b = 2^30, h = 4),
with the runtime knobs the autotuner picks for it (as bench.py times it):
every output of the GPU run is digested and compared with the digests of a
full oracle run stored under tests/golden/ by make_bacterial_digests.py
(oracle only)."""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import synth  # noqa: E402
from digests import digest_outputs  # noqa: E402
from helpers import to_genomes  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = ["bacterial_k25.json", "bacterial_k25_blocked.json", "bacterial_k63.json",
         "bacterial_k100_blocked.json"]


@pytest.fixture(scope="module")
def bacterial():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return synth.bacterial(0)


@pytest.mark.parametrize("case", CASES)
def test_bacterial_full_size_digests(case, bacterial):
    import paper_1602_05856_amd as tp
    path = os.path.join(HERE, "golden", case)
    if not os.path.exists(path):
        pytest.skip("oracle digests %s not generated" % case)
    rec = json.load(open(path))
    k = rec["k"]
    W = 1 if k <= 31 else (2 if k <= 63 else 4)
    flags = tp.TP_FLAG_BLOCKED_FILTER if rec.get("filter") == "blocked" else 0
    print("case: full-size %s k=%d flags=%d" % (case, k, flags), flush=True)
    plan = tp.Plan(to_genomes(bacterial), k, 1 << rec["bloom_log2"], rec["hashes"], flags)
    d_in = plan.upload()
    print("tuned: %s" % plan.autotune(d_in), flush=True)
    plan.run(d_in)
    res = plan.download()
    bloom = plan.debug_bloom()
    c1 = plan.bitmap_positions(plan.debug_candidates())
    plan.close()
    ng = len(bacterial)
    junctions = [res.junctions(g) for g in range(ng)]
    vertex, strand = [], []
    for g in range(ng):
        a, z = res.junction_offset[g], res.junction_offset[g + 1]
        vertex.append(res.vertex[a:z, :W])
        strand.append(res.strand[a:z])
    edges = np.stack([res.edges["genome"].astype(np.uint64), res.edges["from_pos"],
                      res.edges["to_pos"]], axis=1)
    got = digest_outputs(bloom, c1, junctions, vertex, strand, edges, W)
    assert got["counts"] == rec["counts"]
    for key in ("bloom", "c1", "junctions", "vertex", "strand", "edges"):
        assert got[key] == rec[key], key
