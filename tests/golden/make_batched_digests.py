#!/usr/bin/env python3
"""Write the oracle's results on the batched workload (256 independent genome
sets, total size log-uniform in 50 kbp..20 Mbp, 2-10 related genomes each;
k = 31, h = 4, blocked first-pass filter, per set b = the smallest power of
two >= 16 bits per (k+1)-mer position) as SHA-256 digests plus counts, one
entry per set, into batched_k31_blocked.json.

Calls only the CPU oracle (oracle/) and the seeded generator (synth/); the
GPU path never contributes a stored value.  The sets are independent, so
separate single-threaded oracle processes run them in parallel.  Usage:

    python tests/golden/make_batched_digests.py [processes]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

K, H, BITS_PER_EDGE, N_SETS = 31, 4, 16, 256


def one(s):
    import oracle
    import synth
    from digests import digest_outputs, filter_bits
    codes = synth.batched_set(0, s)
    b = filter_bits(codes, K, BITS_PER_EDGE)
    t0 = time.time()
    o = oracle.twopass(codes, K, b, H, blocked=True)
    vx = [oracle.vertex_words(g, K, j) for g, j in zip(codes, o.junctions)]
    edges = oracle.edges(codes, K, o.junctions)
    rec = digest_outputs(o.bloom, o.c1, o.junctions, [w for w, _ in vx], [x for _, x in vx],
                         edges, W=1)
    rec.update({"set": s, "genomes": len(codes), "bases": int(sum(int(c.size) for c in codes)),
                "bloom_bits": b, "oracle_seconds": round(time.time() - t0, 1)})
    return rec


def main(procs):
    t0 = time.time()
    with mp.Pool(procs) as pool:
        recs = []
        for rec in pool.imap_unordered(one, range(N_SETS)):
            recs.append(rec)
            print("set %3d: %d genomes, %.2f Mbp, %d junctions, %.1fs" % (
                rec["set"], rec["genomes"], rec["bases"] / 1e6, rec["counts"]["junctions"],
                rec["oracle_seconds"]), flush=True)
    recs.sort(key=lambda r: r["set"])
    out = {"workload": "batched sets seed 0, %d sets" % N_SETS, "k": K, "hashes": H,
           "filter": "blocked", "bits_per_edge": BITS_PER_EDGE, "sets": recs,
           "oracle_seconds_total": round(sum(r["oracle_seconds"] for r in recs), 1)}
    path = os.path.join(HERE, "batched_k31_blocked.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote %s in %.0fs" % (path, time.time() - t0))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 7)
