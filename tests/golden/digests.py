"""Canonical SHA-256 digests of a junction-finding result, so large results
can be stored and compared without storing them.  Used on oracle output by
make_bacterial_digests.py and on GPU output by the parity tests."""
import hashlib

import numpy as np


def _sha(parts):
    h = hashlib.sha256()
    for p in parts:
        h.update(np.ascontiguousarray(p).tobytes())
    return h.hexdigest()


def digest_outputs(bloom, c1, junctions, vertex, strand, edges, W):
    """bloom: uint32 words; c1, junctions: per-genome uint64 positions;
    vertex: per-genome (n, m) uint64 value words, least significant first
    (m >= W; words beyond W ignored); strand: per-genome uint8; edges: (n, 3)
    uint64 (genome, from, to)."""
    c1 = [np.asarray(x, np.uint64) for x in c1]
    junctions = [np.asarray(x, np.uint64) for x in junctions]
    vx = [np.asarray(v, np.uint64).reshape(len(j), -1)[:, :W]
          for v, j in zip(vertex, junctions)]
    return {
        "bloom": _sha([np.asarray(bloom, np.uint32)]),
        "c1": _sha([np.array([len(x) for x in c1], np.uint64)] + c1),
        "junctions": _sha([np.array([len(x) for x in junctions], np.uint64)] + junctions),
        "vertex": _sha(vx),
        "strand": _sha([np.asarray(s, np.uint8) for s in strand]),
        "edges": _sha([np.asarray(edges, np.uint64).reshape(-1, 3)]),
        "counts": {"c1": int(sum(len(x) for x in c1)),
                   "junctions": int(sum(len(x) for x in junctions)),
                   "edges": int(np.asarray(edges).reshape(-1, 3).shape[0]),
                   "bloom_popcount": int(sum(int(np.unpackbits(np.asarray(bloom, np.uint32)
                                                               .view(np.uint8)).sum())
                                             for _ in [0]))},
    }


def filter_bits(codes, k, bits_per_edge):
    """A workload's filter size: the smallest power of two >= bits_per_edge
    times the (k+1)-mer positions of a genome set (strings are the N-free
    runs), clamped to 2^6..2^40."""
    edges = 0
    for g in codes:
        isn = np.concatenate([[True], np.asarray(g) > 3, [True]])
        runs = np.flatnonzero(isn[1:] != isn[:-1]).reshape(-1, 2)
        edges += int(np.maximum(runs[:, 1] - runs[:, 0] - k, 0).sum())
    b = 64
    while b < (1 << 40) and b < bits_per_edge * edges:
        b <<= 1
    return b
