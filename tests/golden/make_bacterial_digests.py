#!/usr/bin/env python3
"""Write the oracle's results on the full bacterial workload (62 x 5 Mbp,
b = 2^30, h = 4) as SHA-256 digests plus counts, one JSON file per case.

Calls only the CPU oracle (oracle/) and the seeded generator (synth/); the
GPU path never contributes a stored value.  A case is k, optionally followed
by "b" for the blocked first-pass filter.  Usage:

    python tests/golden/make_bacterial_digests.py 25 63 25b 100b
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402
from digests import digest_outputs  # noqa: E402

B_LOG2, H = 30, 4


def main(cases):
    codes = synth.bacterial(0)
    for case in cases:
        blocked = case.endswith("b")
        k = int(case.rstrip("b"))
        t0 = time.time()
        o = oracle.twopass(codes, k, 1 << B_LOG2, H, blocked=blocked)
        t1 = time.time()
        vx = [oracle.vertex_words(g, k, j) for g, j in zip(codes, o.junctions)]
        edges = oracle.edges(codes, k, o.junctions)
        W = 1 if k <= 31 else (2 if k <= 63 else 4)
        rec = digest_outputs(o.bloom, o.c1, o.junctions, [w for w, _ in vx],
                             [s for _, s in vx], edges, W=W)
        rec.update({"workload": "bacterial seed 0, 62 genomes", "k": k, "bloom_log2": B_LOG2,
                    "hashes": H, "filter": "blocked" if blocked else "standard",
                    "oracle_seconds": round(t1 - t0, 1), "stats": o.stats})
        path = os.path.join(HERE, "bacterial_k%d%s.json" % (k, "_blocked" if blocked else ""))
        with open(path, "w") as f:
            json.dump(rec, f, indent=1, sort_keys=True)
        print("wrote", path, rec["counts"], "%.0fs" % (t1 - t0), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["25"])
