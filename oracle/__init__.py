"""TwoPaCo junction-finding oracle -- TEST INFRASTRUCTURE ONLY.

Python marshalling for ``twopaco_oracle.c``: a plain single-threaded CPU
implementation of the paper's definitions (Preliminaries section) and of
Algorithm 2 (Filter-Junctions-Two-Pass, one round) of Minkin, Pham &
Medvedev, arXiv 1602.05856.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the GPU library
and its binding never do.

Genomes are passed as ``numpy.uint8`` arrays of base codes (A=0, C=1, G=2,
T=3, anything above 3 is N).  Positions are 0-based k-mer starts in genome
coordinates.

Parity status: junction positions, vertices and edges are pinned (brute force,
worked example, closed forms, invariants).  Bloom bits and the pass-1
candidate set depend on the hash family, which the paper leaves open: parity
unpinned beyond structural and statistical properties.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "twopaco_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SINGLE_STRAND = 1
BLOCKED = 4   # blocked filter variant: all h bits of an edge in one 64-bit block


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Genome(ctypes.Structure):
    _fields_ = [("codes", ctypes.c_void_p), ("len", ctypes.c_uint64)]


class _PackedGenome(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_void_p), ("n_bases", ctypes.c_uint64),
                ("n_runs", ctypes.c_void_p), ("n_nruns", ctypes.c_uint64)]


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("positions", "marks_pass1", "marks_pass2", "bloom_popcount",
                 "exact_edges", "distinct_edges")]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.or_mix64.restype = U64
        L.or_mix64.argtypes = [U64]
        L.or_bloom_indices.restype = None
        L.or_bloom_indices.argtypes = [P, U32, U64, U32, P]
        L.or_blocked_indices.restype = None
        L.or_blocked_indices.argtypes = [P, U32, U64, U32, U32, P]
        L.or_twopass.restype = I
        L.or_twopass.argtypes = [P, U32, U32, U64, U32, U32, I, P, P, P, P]
        L.or_bruteforce.restype = I
        L.or_bruteforce.argtypes = [P, U32, U32, U32, P]
        L.or_vertex.restype = None
        L.or_vertex.argtypes = [P, U32, U32, P, U64, P, P]
        L.or_edges.restype = ctypes.c_int64
        L.or_edges.argtypes = [P, U32, U32, P, P, U64]
        L.or_sample_status.restype = I
        L.or_sample_status.argtypes = [P, U32, U32, U32, P, P, U64, P, U32]
        L.or_sample_status_packed.restype = I
        L.or_sample_status_packed.argtypes = [P, U32, U32, U32, P, P, U64, P, U32]
        L.or_vertex_masks.restype = I
        L.or_vertex_masks.argtypes = [P, U32, U32, U32, P, U64, P, P, P, U32]
        L.or_vertex_masks_packed.restype = I
        L.or_vertex_masks_packed.argtypes = [P, U32, U32, U32, P, U64, P, P, P, U32]
        L.or_rounds.restype = I
        L.or_rounds.argtypes = [P, U32, U32, U64, U32, U32, U32, P, P, P, P, P, P]
        L.or_partition.restype = None
        L.or_partition.argtypes = [P, U32, P]
        L.or_subrange.restype = U32
        L.or_subrange.argtypes = [P, U32]
        _lib_handle = L
    return _lib_handle


def _genome_array(genomes):
    gs = [np.ascontiguousarray(g, dtype=np.uint8) for g in genomes]
    arr = (_Genome * max(1, len(gs)))()
    for i, g in enumerate(gs):
        arr[i].codes = g.ctypes.data if g.size else None
        arr[i].len = g.size
    return gs, arr


def _mark_arrays(gs):
    marks = [np.zeros(max(1, g.size), dtype=np.uint8) for g in gs]
    ptrs = (ctypes.c_void_p * max(1, len(gs)))(*[m.ctypes.data for m in marks])
    return marks, ptrs


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, rc))


def mix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood 2014)."""
    return int(_lib().or_mix64(ctypes.c_uint64(x & (2**64 - 1))))


def _words(value: int) -> np.ndarray:
    return np.array([(value >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)


def bloom_indices(value: int, k: int, b: int, h: int) -> list[int]:
    """Bit indices of the (k+1)-mer with the given value in a b-bit filter."""
    out = np.zeros(h, dtype=np.uint64)
    w = _words(value)
    _lib().or_bloom_indices(w.ctypes.data, k, b, h, out.ctypes.data)
    return [int(v) for v in out]


def blocked_indices(edge_codes, k: int, b: int, h: int, single_strand=False) -> list[int]:
    """Blocked-filter bit indices of the (k+1)-mer given as base codes."""
    e = np.ascontiguousarray(edge_codes, dtype=np.uint8)
    assert e.size == k + 1
    out = np.zeros(h, dtype=np.uint64)
    _lib().or_blocked_indices(e.ctypes.data, k, b, h, SINGLE_STRAND if single_strand else 0,
                              out.ctypes.data)
    return [int(v) for v in out]


def _flags(single_strand, blocked):
    return (SINGLE_STRAND if single_strand else 0) | (BLOCKED if blocked else 0)


@dataclass
class TwoPass:
    bloom: np.ndarray          # uint32[b/32], the first-pass filter F
    c1: list                   # per genome: sorted positions marked after pass 1
    junctions: list            # per genome: sorted positions marked after pass 2 (= J)
    stats: dict


def twopass(genomes, k, b, h, single_strand=False, with_distinct=False,
            blocked=False) -> TwoPass:
    """Algorithm 2 with one round, all positions initially marked; the first
    pass uses the standard or the blocked filter layout."""
    gs, arr = _genome_array(genomes)
    c1, p1 = _mark_arrays(gs)
    c2, p2 = _mark_arrays(gs)
    bloom = np.zeros(b // 32, dtype=np.uint32)
    st = _Stats()
    rc = _lib().or_twopass(ctypes.addressof(arr), len(gs), k, b, h,
                           _flags(single_strand, blocked), int(with_distinct),
                           bloom.ctypes.data, ctypes.addressof(p1), ctypes.addressof(p2),
                           ctypes.addressof(st))
    _check(rc, "twopass")
    stats = {n: int(getattr(st, n)) for n, _ in _Stats._fields_}
    return TwoPass(bloom=bloom,
                   c1=[np.flatnonzero(m[:g.size]).astype(np.uint64) for m, g in zip(c1, gs)],
                   junctions=[np.flatnonzero(m[:g.size]).astype(np.uint64) for m, g in zip(c2, gs)],
                   stats=stats)


Q = 1024   # hash subranges of the partition heuristic (Multiple Rounds section)


@dataclass
class Rounds(TwoPass):
    counters: np.ndarray = None   # uint64[Q], the census e_i
    bounds: np.ndarray = None     # uint32[l + 1], class c = subranges [bounds[c], bounds[c+1])


def rounds(genomes, k, b, h, l, single_strand=False, blocked=False) -> Rounds:
    """Algorithm 3 with l rounds: ``c1`` and ``junctions`` are the unions of the
    rounds' first- and second-pass marks, ``bloom`` the last round's filter."""
    gs, arr = _genome_array(genomes)
    c1, p1 = _mark_arrays(gs)
    c2, p2 = _mark_arrays(gs)
    bloom = np.zeros(b // 32, dtype=np.uint32)
    counters = np.zeros(Q, dtype=np.uint64)
    bounds = np.zeros(l + 1, dtype=np.uint32)
    st = _Stats()
    rc = _lib().or_rounds(ctypes.addressof(arr), len(gs), k, b, h, _flags(single_strand, blocked),
                          l, bloom.ctypes.data, ctypes.addressof(p1), ctypes.addressof(p2),
                          ctypes.addressof(st), counters.ctypes.data, bounds.ctypes.data)
    _check(rc, "rounds")
    stats = {n: int(getattr(st, n)) for n, _ in _Stats._fields_}
    return Rounds(bloom=bloom,
                  c1=[np.flatnonzero(m[:g.size]).astype(np.uint64) for m, g in zip(c1, gs)],
                  junctions=[np.flatnonzero(m[:g.size]).astype(np.uint64) for m, g in zip(c2, gs)],
                  stats=stats, counters=counters, bounds=bounds)


def partition(counters, l) -> np.ndarray:
    """Class bounds (l + 1 subrange indices) of the greedy partition."""
    e = np.ascontiguousarray(counters, dtype=np.uint64)
    assert e.size == Q
    out = np.zeros(l + 1, dtype=np.uint32)
    _lib().or_partition(e.ctypes.data, l, out.ctypes.data)
    return out


def subrange(value: int, k: int) -> int:
    """Hash subrange (0..Q-1) of a normalised k-mer value."""
    w = _words(value)
    return int(_lib().or_subrange(w.ctypes.data, k))


def bruteforce(genomes, k, single_strand=False) -> list:
    """J(S,k) from the definitions on the comprehensive graph."""
    gs, arr = _genome_array(genomes)
    j, pj = _mark_arrays(gs)
    rc = _lib().or_bruteforce(ctypes.addressof(arr), len(gs), k,
                              SINGLE_STRAND if single_strand else 0, ctypes.addressof(pj))
    _check(rc, "bruteforce")
    return [np.flatnonzero(m[:g.size]).astype(np.uint64) for m, g in zip(j, gs)]


def vertex_words(genome, k, positions, single_strand=False):
    """(words, strand): the normalised k-mer at each position as four 64-bit
    words (least significant first), and its strand."""
    gs, arr = _genome_array([genome])
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    words = np.zeros((max(1, pos.size), 4), dtype=np.uint64)
    strand = np.zeros(pos.size, dtype=np.uint8)
    if pos.size:
        _lib().or_vertex(ctypes.addressof(arr), k, SINGLE_STRAND if single_strand else 0,
                         pos.ctypes.data, pos.size, words.ctypes.data, strand.ctypes.data)
    return words[:pos.size].copy(), strand


def vertices(genome, k, positions, single_strand=False):
    """(lo, hi, strand) of the normalised k-mer at each position (the two low
    words of the value; see vertex_words for k > 63)."""
    words, strand = vertex_words(genome, k, positions, single_strand)
    return words[:, 0].copy(), words[:, 1].copy(), strand


def edges(genomes, k, junctions) -> np.ndarray:
    """Compacted edges (genome, from, to), one per pair of consecutive
    junctions of one string, in genome then position order."""
    gs, arr = _genome_array(genomes)
    marks, ptrs = _mark_arrays(gs)
    for m, js in zip(marks, junctions):
        m[np.asarray(js, dtype=np.int64)] = 1
    total = sum(len(js) for js in junctions)
    out = np.zeros((max(1, total), 3), dtype=np.uint64)
    n = _lib().or_edges(ctypes.addressof(arr), len(gs), k, ctypes.addressof(ptrs),
                        out.ctypes.data, out.shape[0])
    _check(0 if n >= 0 else int(n), "edges")
    assert n <= out.shape[0]
    return out[:n].copy()


def _threads(threads):
    if threads:
        return int(threads)
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _packed_array(packed_genomes):
    """(keep-alive list, ctypes array) of (packed bytes, n_bases, N runs) genomes."""
    keep, arr = [], (_PackedGenome * max(1, len(packed_genomes)))()
    for i, (pk, n, runs) in enumerate(packed_genomes):
        pk = np.ascontiguousarray(pk, dtype=np.uint8)
        rs = np.ascontiguousarray(np.asarray(runs, dtype=np.uint64).reshape(-1, 2))
        keep += [pk, rs]
        arr[i].packed = pk.ctypes.data if pk.size else None
        arr[i].n_bases = int(n)
        arr[i].n_runs = rs.ctypes.data if rs.size else None
        arr[i].n_nruns = rs.shape[0]
    return keep, arr


def vertex_masks(genomes, k, values, single_strand=False, threads=None, packed=False):
    """(in_mask, out_mask, sentinel) of the given vertices (literal k-mer values,
    Python ints) of the comprehensive graph, by the definitions: bit c of
    in_mask is set when c.v is an edge, bit c of out_mask when v.c is one.
    ``genomes`` are code arrays, or with ``packed`` (packed bytes, n_bases,
    N runs) tuples."""
    vw = np.zeros((max(1, len(values)), 4), dtype=np.uint64)
    for i, v in enumerate(values):
        vw[i] = _words(int(v))
    n = len(values)
    inm, outm, sent = (np.zeros(max(1, n), dtype=np.uint8) for _ in range(3))
    flags = SINGLE_STRAND if single_strand else 0
    if packed:
        keep, arr = _packed_array(genomes)
        fn = _lib().or_vertex_masks_packed
    else:
        keep, arr = _genome_array(genomes)
        fn = _lib().or_vertex_masks
    rc = fn(ctypes.addressof(arr), len(genomes), k, flags, vw.ctypes.data, n, inm.ctypes.data,
            outm.ctypes.data, sent.ctypes.data, _threads(threads))
    del keep
    _check(rc, "vertex_masks")
    return inm[:n], outm[:n], sent[:n]


def sample_status(genomes, k, samp_genome, samp_pos, single_strand=False, threads=None,
                  packed=False) -> np.ndarray:
    """Junction status (by the definitions) of the sampled positions: a
    sentinel, or more than one in- or out-edge in the comprehensive graph.
    ``genomes`` are code arrays, or with ``packed`` (packed bytes, n_bases,
    N runs) tuples."""
    sg = np.ascontiguousarray(samp_genome, dtype=np.uint32)
    sp = np.ascontiguousarray(samp_pos, dtype=np.uint64)
    out = np.zeros(max(1, sp.size), dtype=np.uint8)
    flags = SINGLE_STRAND if single_strand else 0
    if packed:
        keep, arr = _packed_array(genomes)
        fn = _lib().or_sample_status_packed
    else:
        keep, arr = _genome_array(genomes)
        fn = _lib().or_sample_status
    rc = fn(ctypes.addressof(arr), len(genomes), k, flags, sg.ctypes.data, sp.ctypes.data,
            sp.size, out.ctypes.data, _threads(threads))
    del keep
    _check(rc, "sample_status")
    return out[:sp.size]
