"""Seeded synthetic genomes.

The input generator shared by the oracle tests and the GPU tests and
benchmarks.  It draws bases, repeats and mutations and formats them; it holds
none of the junction-finding arithmetic.

The paper's datasets (62 E. coli, human assemblies, primates) are not
available, so these generators stand in for their shapes: closely related
complete genomes derived from one random base, with SNPs, short indels,
interspersed repeat families and (optionally) runs of N.

Genomes are ``numpy.uint8`` arrays of base codes A=0, C=1, G=2, T=3 and
N=4.  ``pack`` turns one into the library's input format: 2 bits per base,
base j in byte j>>2 at bits 2*(j&3), N stored as 0 and listed separately as
(start, length) runs.

Every stream is a PCG64 generator keyed by a SeedSequence of
(MASTER, workload id, seed, sub-stream ...), so a workload is the same on any
machine with the same numpy.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

MASTER = 0x1602058560


def rng(*keys: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER, *keys])))


def random_bases(r: np.random.Generator, n: int) -> np.ndarray:
    return r.integers(0, 4, int(n), dtype=np.uint8)


def substitute(r: np.random.Generator, seq: np.ndarray, rate: float) -> np.ndarray:
    """Each base independently with probability ``rate`` becomes one of the
    other three, chosen uniformly."""
    out = seq.copy()
    hit = np.flatnonzero((r.random(seq.size) < rate) & (seq < 4))
    out[hit] = (out[hit] + r.integers(1, 4, hit.size, dtype=np.uint8)) % 4
    return out


def indels(r: np.random.Generator, seq: np.ndarray, rate: float, maxlen: int = 10) -> np.ndarray:
    """round(rate*len) events at uniform offsets, half insertions of random
    bases and half deletions, each of length uniform in 1..maxlen."""
    n_ev = int(round(rate * seq.size))
    if n_ev == 0 or seq.size == 0:
        return seq.copy()
    pos = np.sort(r.integers(0, seq.size, n_ev))
    ins = r.random(n_ev) < 0.5
    lens = r.integers(1, maxlen + 1, n_ev)
    pool = random_bases(r, int(lens[ins].sum()))
    pieces, cur, used = [], 0, 0
    for p, is_ins, ln in zip(pos.tolist(), ins.tolist(), lens.tolist()):
        if p < cur:
            continue
        pieces.append(seq[cur:p])
        if is_ins:
            pieces.append(pool[used:used + ln])
            used += ln
            cur = p
        else:
            cur = p + ln
    pieces.append(seq[cur:])
    return np.concatenate(pieces)


def plant_repeats(r: np.random.Generator, seq: np.ndarray, family_len: int, copies: int,
                  divergence: float) -> np.ndarray:
    """Overwrite ``copies`` uniform offsets of ``seq`` with copies of one
    random family consensus, each copy with ``divergence`` substitutions."""
    if family_len > seq.size:
        return seq
    fam = random_bases(r, family_len)
    offs = r.integers(0, seq.size - family_len + 1, copies)
    for off in offs.tolist():
        seq[off:off + family_len] = substitute(r, fam, divergence)
    return seq


def n_runs(r: np.random.Generator, seq: np.ndarray, count: int, lo: int, hi: int) -> np.ndarray:
    """Replace ``count`` uniform stretches of length U[lo,hi] with N."""
    out = seq.copy()
    for _ in range(count):
        ln = int(r.integers(lo, hi + 1))
        if ln >= out.size:
            continue
        off = int(r.integers(0, out.size - ln + 1))
        out[off:off + ln] = 4
    return out


def pack(codes: np.ndarray):
    """(packed uint8[ceil(n/4)], n_runs uint64[m,2]) for one genome."""
    codes = np.asarray(codes, dtype=np.uint8)
    n = codes.size
    isn = codes > 3
    c = np.where(isn, 0, codes).astype(np.uint8)
    c = np.concatenate([c, np.zeros((-n) % 4, np.uint8)]).reshape(-1, 4)
    packed = (c[:, 0] | (c[:, 1] << 2) | (c[:, 2] << 4) | (c[:, 3] << 6)).astype(np.uint8)
    if isn.any():
        d = np.diff(np.concatenate([[0], isn.astype(np.int8), [0]]))
        starts = np.flatnonzero(d == 1)
        ends = np.flatnonzero(d == -1)
        runs = np.stack([starts, ends - starts], axis=1).astype(np.uint64)
    else:
        runs = np.zeros((0, 2), dtype=np.uint64)
    return packed, runs


def reverse_complement(codes: np.ndarray) -> np.ndarray:
    codes = np.asarray(codes, dtype=np.uint8)
    out = codes[::-1].copy()
    ok = out < 4
    out[ok] = 3 - out[ok]
    return out


# ---------------------------------------------------------------- workloads

def plain_small(seed: int = 0):
    """4 genomes of 100 kbp.  Genome 0 is uniform i.i.d. with 20 copies of one
    300 bp repeat at 5% divergence; genomes 1-3 are copies of it with 1% SNPs
    and 0.1% indels of length 1-10.  (k=25, b=2^24, h=3.)"""
    r = rng(1, seed)
    g0 = random_bases(r, 100_000)
    plant_repeats(r, g0, 300, 20, 0.05)
    gs = [g0]
    for i in range(3):
        ri = rng(1, seed, 1 + i)
        gs.append(indels(ri, substitute(ri, g0, 0.01), 0.001))
    return gs


def bacterial(seed: int = 0, n_genomes: int = 62, length: int = 5_000_000):
    """62 genomes of ~5 Mbp derived from one random base genome (not itself
    included): per genome U[0.5%,2%] SNPs and 0.2% indels; the base carries 50
    repeat families of U[1,5] kbp, two copies each at 5% divergence.
    (k=25 and k=63, b=2^30, h=4.)"""
    r = rng(2, seed)
    base = random_bases(r, length)
    for _ in range(50):
        plant_repeats(r, base, int(r.integers(1000, 5001)), 2, 0.05)
    gs = []
    for i in range(n_genomes):
        ri = rng(2, seed, 1 + i)
        d = float(ri.uniform(0.005, 0.02))
        gs.append(indels(ri, substitute(ri, base, d), 0.002))
    return gs


def batched_sets(seed: int = 0, n_sets: int = 256, lo: float = 50e3, hi: float = 20e6):
    """Independent genome sets of uneven size: total size log-uniform in
    [lo, hi], 2-10 genomes per set at 1% SNPs + 0.1% indels from a set base
    with 5% repeat content (10 families of U[300,3000] bp at 5% divergence).
    (k=31, b = 2^ceil(log2(16 * (k+1)-mers)) per set, h=4.)"""
    return [batched_set(seed, s, lo, hi) for s in range(n_sets)]


def batched_set(seed: int, s: int, lo: float = 50e3, hi: float = 20e6):
    """Set ``s`` of ``batched_sets(seed)``, generated on its own (its size and
    genome count come from the workload's stream, drawn in set order)."""
    r = rng(3, seed)
    for _ in range(s + 1):
        total = float(math.exp(r.uniform(math.log(lo), math.log(hi))))
        g = int(r.integers(2, 11))
    return genome_set(rng(3, seed, 1 + s), int(total / g), g)


# Serving workload: request classes (name, share, total set size range in
# bases, k) and how many distinct sets the pool holds per class.
SERVE_CLASSES = (
    ("small", 0.70, (1e6, 5e6), 25),
    ("medium", 0.25, (50e6, 200e6), 31),
    ("large", 0.05, (1e9, 3e9), 63),
)
SERVE_POOL = {"small": 8, "medium": 3, "large": 3}


def serving_entries(seed: int = 0):
    """[(class name, k, index, genome length, genome count)] of the serving
    pool: per class, set totals log-uniform in its range and 2-10 genomes."""
    r = rng(5, seed)
    out = []
    for name, _, (lo, hi), k in SERVE_CLASSES:
        for i in range(SERVE_POOL[name]):
            total = float(math.exp(r.uniform(math.log(lo), math.log(hi))))
            g = int(r.integers(2, 11))
            out.append((name, k, i, int(total / g), g))
    return out


def serving_set(seed: int, entry):
    """Genomes (base codes) of one serving-pool entry, built as the batched
    workload's sets are."""
    name, k, i, glen, g = entry
    ci = [c[0] for c in SERVE_CLASSES].index(name)
    return genome_set(rng(5, seed, 1 + ci, i), glen, g)


def genome_set(r: np.random.Generator, genome_len: int, n_genomes: int,
               divergence: float = 0.01, repeat_frac: float = 0.05):
    base = random_bases(r, genome_len)
    fams = 10
    for _ in range(fams):
        flen = int(r.integers(300, 3001))
        copies = max(1, int(round(repeat_frac * genome_len / fams / flen)))
        plant_repeats(r, base, flen, copies, 0.05)
    return [indels(r, substitute(r, base, divergence), divergence / 10) for _ in range(n_genomes)]


def random_genomes(seed: int, n: int, lo: int, hi: int, alphabet: int = 4, n_frac: float = 0.0):
    """Small random genomes for edge-case tests: lengths U[lo,hi], bases
    uniform over the first ``alphabet`` codes, optional N stretches."""
    r = rng(9, seed)
    gs = []
    for _ in range(n):
        ln = int(r.integers(lo, hi + 1))
        g = r.integers(0, alphabet, ln, dtype=np.uint8)
        if n_frac > 0 and ln > 0:
            g[r.random(ln) < n_frac] = 4
        gs.append(g)
    return gs


# ------------------------------------------------ primate-scale (C generator)

_HERE = os.path.dirname(os.path.abspath(__file__))
_PRIMATE_SRC = os.path.join(_HERE, "primate.c")
_PRIMATE_LIB = os.path.join(_HERE, "libsynth.so")
_primate_handle = None


def build_native(force: bool = False) -> str:
    """Compile the C generator with gcc into ``synth/libsynth.so``."""
    if (force or not os.path.exists(_PRIMATE_LIB)
            or os.path.getmtime(_PRIMATE_LIB) < os.path.getmtime(_PRIMATE_SRC)):
        tmp = _PRIMATE_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _PRIMATE_SRC, "-lm"])
        os.replace(tmp, _PRIMATE_LIB)
    return _PRIMATE_LIB


def _native():
    global _primate_handle
    if _primate_handle is None:
        L = ctypes.CDLL(build_native())
        U64, P = ctypes.c_uint64, ctypes.c_void_p
        L.syn_primate_base_len.restype = U64
        L.syn_primate_base_len.argtypes = [ctypes.c_double]
        L.syn_primate_base.restype = None
        L.syn_primate_base.argtypes = [U64, ctypes.c_double, P]
        L.syn_primate_genome_cap.restype = U64
        L.syn_primate_genome_cap.argtypes = [U64, ctypes.c_uint32]
        L.syn_primate_genome.restype = U64
        L.syn_primate_genome.argtypes = [P, U64, U64, ctypes.c_double, ctypes.c_uint32, P, U64]
        L.syn_pack.restype = U64
        L.syn_pack.argtypes = [P, U64, P, P, U64]
        _primate_handle = L
    return _primate_handle


def primate(seed: int = 0, scale: float = 1.0, n_genomes: int = 8, packed: bool = False,
            threads: int = 8):
    """Primate-scale workload: 8 genomes of 3 Gbp (times ``scale``) from one
    random base with 45%-style interspersed repeats (1e6 copies of a 300 bp
    family and 1e5 of a 6 kbp family at 10-20% divergence), per-genome SNPs
    at 0.5% + g * 3.5% / 7 (pairwise 1-8%), indels at a tenth of that and 300
    N runs of 1-10 kbp (recipe in primate.c).  k=25, b=2^36, h=5.

    Returns base-code arrays, or with ``packed`` (packed bytes, n_bases, N
    runs) per genome without materialising the codes of all genomes at once."""
    import concurrent.futures

    L = _native()
    s = (MASTER + 4 + (int(seed) << 8)) & ((1 << 64) - 1)
    n = int(L.syn_primate_base_len(float(scale)))
    base = np.empty(n, dtype=np.uint8)
    L.syn_primate_base(s, float(scale), base.ctypes.data)

    def one(g):
        cap = int(L.syn_primate_genome_cap(n, g))
        out = np.empty(cap, dtype=np.uint8)
        m = int(L.syn_primate_genome(base.ctypes.data, n, s, float(scale), g, out.ctypes.data,
                                     cap))
        if m == 0:
            raise RuntimeError("primate generator: genome %d exceeded its capacity" % g)
        if not packed:
            return out[:m].copy()
        pk = np.empty((m + 3) // 4, dtype=np.uint8)
        max_runs = 4096
        runs = np.empty((max_runs, 2), dtype=np.uint64)
        nr = int(L.syn_pack(out.ctypes.data, m, pk.ctypes.data, runs.ctypes.data, max_runs))
        if nr > max_runs:
            raise RuntimeError("primate generator: too many N runs")
        del out
        return pk, m, runs[:nr].copy()

    with concurrent.futures.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(one, range(n_genomes)))
