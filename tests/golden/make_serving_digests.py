#!/usr/bin/env python3
"""Write the oracle's results on the small and medium sets of the serving
pool (synth.serving_entries: 1-5 Mbp sets at k = 25, 50-200 Mbp sets at
k = 31; h = 4, blocked first-pass filter, b = the smallest power of two
>= 16 bits per (k+1)-mer position) as SHA-256 digests plus counts, into
serving_pool.json.  The 1-3 Gbp sets at k = 63 are checked by sampled
junction status at test time instead.

Calls only the CPU oracle (oracle/) and the seeded generator (synth/); the
GPU path never contributes a stored value.  Sets run in parallel processes.
Usage:  python tests/golden/make_serving_digests.py [processes]
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

H, BITS_PER_EDGE = 4, 16


def one(entry):
    import oracle
    import synth
    from digests import digest_outputs, filter_bits
    name, k, i, glen, g = entry
    codes = synth.serving_set(0, entry)
    b = filter_bits(codes, k, BITS_PER_EDGE)
    t0 = time.time()
    o = oracle.twopass(codes, k, b, H, blocked=True)
    vx = [oracle.vertex_words(c, k, j) for c, j in zip(codes, o.junctions)]
    edges = oracle.edges(codes, k, o.junctions)
    W = 1 if k <= 31 else (2 if k <= 63 else 4)
    rec = digest_outputs(o.bloom, o.c1, o.junctions, [w for w, _ in vx], [x for _, x in vx],
                         edges, W=W)
    rec.update({"class": name, "index": i, "k": k, "genomes": len(codes),
                "bases": int(sum(int(c.size) for c in codes)), "bloom_bits": b,
                "oracle_seconds": round(time.time() - t0, 1)})
    return rec


def main(procs):
    import synth
    entries = [e for e in synth.serving_entries(0) if e[0] != "large"]
    entries.sort(key=lambda e: -e[3] * e[4])  # longest first
    t0 = time.time()
    with mp.Pool(procs) as pool:
        recs = []
        for rec in pool.imap_unordered(one, entries):
            recs.append(rec)
            print("%s %d: %.1f Mbp, %d junctions, %.0fs" % (
                rec["class"], rec["index"], rec["bases"] / 1e6, rec["counts"]["junctions"],
                rec["oracle_seconds"]), flush=True)
    recs.sort(key=lambda r: (r["class"], r["index"]))
    out = {"workload": "serving pool seed 0 (small and medium classes)", "hashes": H,
           "filter": "blocked", "bits_per_edge": BITS_PER_EDGE, "sets": recs}
    path = os.path.join(HERE, "serving_pool.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote %s in %.0fs" % (path, time.time() - t0))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4)
