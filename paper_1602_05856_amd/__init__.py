"""Python binding of ``libtwopaco.so``, the gfx950 TwoPaCo junction-finding
library (C ABI in ``include/twopaco.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory (the packed input buffer) and the
stream.  There is no CPU fallback: importing works anywhere, but every call
that needs the library raises when ``libtwopaco.so`` is missing or cannot be
loaded.

Genome inputs are ``Genome`` records in the library's format: ``packed`` is a
``numpy.uint8`` array with base j (A=0 C=1 G=2 T=3) in byte j>>2 at bits
2*(j&3), ``n_bases`` the length including N, ``n_runs`` an (m, 2) uint64
array of (start, length) N runs.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; TWOPACO_LIB may name another build of the same sources
LIB_PATH = os.environ.get("TWOPACO_LIB") or os.path.join(_HERE, "libtwopaco.so")

TP_OK, TP_EINVAL, TP_ENOMEM, TP_EOVERFLOW, TP_EDEVICE, TP_ESTATE = 0, -1, -2, -3, -4, -5
TP_ETIMEOUT = -6
TP_EPENDING = -7
TP_WS_TABLE_OVERFLOW, TP_WS_OUTPUT_OVERFLOW, TP_WS_INTERNAL = 1, 2, 4
TP_FLAG_SINGLE_STRAND = 1
TP_FLAG_PASS1_ONLY = 2
TP_FLAG_BLOCKED_FILTER = 4

_STATUS = {TP_EINVAL: "TP_EINVAL", TP_ENOMEM: "TP_ENOMEM", TP_EOVERFLOW: "TP_EOVERFLOW",
           TP_EDEVICE: "TP_EDEVICE", TP_ESTATE: "TP_ESTATE", TP_ETIMEOUT: "TP_ETIMEOUT",
           TP_EPENDING: "TP_EPENDING"}


class TwoPaCoError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__("%s failed: %s (%s)" % (where, message, _STATUS.get(status, status)))
        self.status = status


class tp_genome(ctypes.Structure):
    _fields_ = [("packed", ctypes.c_void_p), ("n_bases", ctypes.c_uint64),
                ("n_runs", ctypes.c_void_p), ("n_nruns", ctypes.c_uint64)]


class tp_edge(ctypes.Structure):
    _fields_ = [("genome", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("from_pos", ctypes.c_uint64), ("to_pos", ctypes.c_uint64)]


class tp_stats(ctypes.Structure):
    _fields_ = [("positions", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("junctions", ctypes.c_uint64), ("edges", ctypes.c_uint64),
                ("bloom_popcount", ctypes.c_uint64), ("table_capacity", ctypes.c_uint64),
                ("table_keys", ctypes.c_uint64), ("distinct_estimate", ctypes.c_uint64),
                ("table_attempts", ctypes.c_uint32), ("sentinels", ctypes.c_uint32),
                ("edge_positions", ctypes.c_uint64), ("fill_atomics", ctypes.c_uint64),
                ("query_probes", ctypes.c_uint64), ("table_probes", ctypes.c_uint64),
                ("ms_sentinels", ctypes.c_float), ("ms_fill", ctypes.c_float),
                ("ms_query", ctypes.c_float), ("ms_record", ctypes.c_float),
                ("ms_decide", ctypes.c_float), ("ms_pass1", ctypes.c_float),
                ("ms_pass2", ctypes.c_float), ("ms_compact", ctypes.c_float),
                ("ms_total", ctypes.c_float), ("rounds", ctypes.c_uint32),
                ("fill_chunks", ctypes.c_uint32), ("record_passes", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class tp_result(ctypes.Structure):
    _fields_ = [("n_genomes", ctypes.c_uint32), ("kmer_words", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("n_junctions", ctypes.c_uint64),
                ("junction_offset", ctypes.c_void_p), ("junction_pos", ctypes.c_void_p),
                ("vertex", ctypes.c_void_p), ("strand", ctypes.c_void_p),
                ("n_edges", ctypes.c_uint64), ("edges", ctypes.c_void_p),
                ("stats", tp_stats)]


class tp_set(ctypes.Structure):
    _fields_ = [("genomes", ctypes.c_void_p), ("n_genomes", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("bloom_bits", ctypes.c_uint64)]


class tp_config(ctypes.Structure):
    _fields_ = [("wg_per_cu", ctypes.c_uint32 * 4), ("tile_order", ctypes.c_uint32),
                ("table_load", ctypes.c_float), ("graphs", ctypes.c_uint32),
                ("pass2_slabs", ctypes.c_uint32), ("fill_dedup", ctypes.c_uint32),
                ("table_shape", ctypes.c_uint32), ("chunk_tiles", ctypes.c_uint32),
                ("fill_binned", ctypes.c_uint32), ("bin_chunk_tiles", ctypes.c_uint32),
                ("bloom_bits_per_edge", ctypes.c_uint32), ("tile_queue", ctypes.c_uint32),
                ("record_binned", ctypes.c_uint32), ("table_budget", ctypes.c_uint64),
                ("record_passes", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class tp_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("workers", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("batch_max_bases", ctypes.c_uint64),
                ("batch_total_bases", ctypes.c_uint64), ("wg_per_cu", ctypes.c_uint32),
                ("express_workers", ctypes.c_uint32), ("express_cus", ctypes.c_uint32),
                ("table_budget_mib", ctypes.c_uint32)]


class tp_job_info(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("start_s", ctypes.c_double),
                ("end_s", ctypes.c_double), ("batch_jobs", ctypes.c_uint32),
                ("worker", ctypes.c_uint32), ("bases", ctypes.c_uint64),
                ("layout_ms", ctypes.c_float), ("upload_ms", ctypes.c_float),
                ("run_ms", ctypes.c_float), ("download_ms", ctypes.c_float)]


class tp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("running", ctypes.c_uint64),
                ("held_bytes", ctypes.c_uint64), ("peak_held_bytes", ctypes.c_uint64)]


class tp_device_outputs(ctypes.Structure):
    _fields_ = [("n_junctions", ctypes.c_uint64), ("junction_offset", ctypes.c_void_p),
                ("junction_pos", ctypes.c_void_p), ("vertex", ctypes.c_void_p),
                ("strand", ctypes.c_void_p), ("n_edges", ctypes.c_uint64),
                ("edges", ctypes.c_void_p), ("candidates", ctypes.c_void_p),
                ("junction_bits", ctypes.c_void_p), ("bloom", ctypes.c_void_p)]


class tp_ws_counts(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint64), ("positions", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64), ("junctions", ctypes.c_uint64),
                ("edges", ctypes.c_uint64), ("table_keys", ctypes.c_uint64),
                ("bloom_popcount", ctypes.c_uint64), ("reserved", ctypes.c_uint64 * 9)]


class tp_ws_layout(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("output_bytes", ctypes.c_uint64),
                ("max_junctions", ctypes.c_uint64), ("max_edges", ctypes.c_uint64),
                ("table_slots", ctypes.c_uint64), ("kmer_words", ctypes.c_uint32),
                ("rounds", ctypes.c_uint32),
                ("off_counts", ctypes.c_uint64), ("off_joff", ctypes.c_uint64),
                ("off_pos", ctypes.c_uint64), ("off_vertex", ctypes.c_uint64),
                ("off_strand", ctypes.c_uint64), ("off_edges", ctypes.c_uint64),
                ("ws_off_candidates", ctypes.c_uint64), ("ws_off_junction_bits", ctypes.c_uint64),
                ("ws_off_bloom", ctypes.c_uint64), ("ws_off_set_counters", ctypes.c_uint64)]


WS_COUNT_FIELDS = ("status", "positions", "candidates", "junctions", "edges", "table_keys",
                   "bloom_popcount")

EDGE_DTYPE = np.dtype([("genome", "<u4"), ("flags", "<u4"), ("from_pos", "<u8"),
                       ("to_pos", "<u8")])

# name -> (restype, argtypes); every symbol include/twopaco.h declares
P, U32, U64, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
SIGNATURES = {
    "twopaco_build": (I, [P, U32, U32, U64, U32, P]),
    "twopaco_build_ex": (I, [P, U32, U32, U64, U32, U32, P]),
    "twopaco_result_free": (None, [P]),
    "twopaco_last_error": (ctypes.c_char_p, []),
    "tp_plan_create": (I, [P, U32, U32, U64, U32, U32, P]),
    "tp_plan_destroy": (None, [P]),
    "tp_plan_input_bytes": (U64, [P]),
    "tp_plan_genome_offset": (U64, [P, U32]),
    "tp_plan_bitmap_words": (U64, [P]),
    "tp_plan_strings": (U64, [P]),
    "tp_plan_upload": (I, [P, P, P, P]),
    "tp_run": (I, [P, P, P]),
    "tp_get_stats": (I, [P, P]),
    "tp_get_device_outputs": (I, [P, P]),
    "tp_download": (I, [P, P, P]),
    "tp_debug_bloom": (I, [P, P, U64]),
    "tp_debug_candidates": (I, [P, P, U64]),
    "tp_batch_create": (I, [P, U32, U32, U32, U32, P]),
    "tp_plan_sets": (U32, [P]),
    "tp_plan_set_first_genome": (U32, [P, U32]),
    "tp_plan_bloom_words": (U64, [P]),
    "tp_plan_set_bloom_offset": (U64, [P, U32]),
    "tp_plan_set_bloom_bits": (U64, [P, U32]),
    "tp_batch_upload": (I, [P, P, P, P]),
    "tp_get_set_stats": (I, [P, U32, P]),
    "tp_download_set": (I, [P, U32, P, P]),
    "tp_debug_set_bloom": (I, [P, U32, P, U64]),
    "tp_bloom_bits_for": (U64, [P, U32, U32, ctypes.c_double]),
    "tp_plan_get_config": (I, [P, P]),
    "tp_plan_set_config": (I, [P, P]),
    "tp_autotune": (I, [P, P, P, ctypes.c_char_p, P]),
    "tp_plan_set_rounds": (I, [P, U32]),
    "tp_plan_rounds": (U32, [P]),
    "tp_plan_class_bounds": (I, [P, U32, P, U32]),
    "tp_server_create": (I, [P, P]),
    "tp_server_submit": (I, [P, P, U32, U32, U64, U32, U32, P]),
    "tp_server_wait": (I, [P, U64, ctypes.c_int64, P, P]),
    "tp_server_get_stats": (I, [P, P]),
    "tp_server_destroy": (None, [P]),
    "tp_server_poll": (I, [P, U64, P, P]),
    "tp_build_batch": (I, [P, U32, U32, U32, U32, P]),
    "tp_debug_table": (I, [P, U32, P, P, U64, P]),
    "tp_plan_workspace_layout": (I, [P, ctypes.c_double, ctypes.c_double, P]),
    "tp_plan_workspace_bytes": (U64, [P]),
    "tp_plan_prepare_workspace": (I, [P, P, P]),
    "tp_run_ws": (I, [P, P, P, P, P]),
    "tp_run_noalloc": (I, [P, P, P, P]),
    "tp_bench_random_access": (I, [P, U64, U64, U32, U64, P, P, P]),
}

NOALLOC_WORKSPACE_MAX = 64 << 20  # TP_NOALLOC_WORKSPACE_MAX

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises when it has not been built."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (needed as libamdhip64.so, with the
        # same soname libamdhip64.so.7 as the system one this library links).
        # Loaded first, it satisfies this library's dependency and the process
        # has one runtime; loaded after, torch would bring a second runtime,
        # and the two do not share the device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtwopaco.so is not built (run __graft_entry__.build() or "
                              "python paper_1602_05856_amd/_build.py)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().twopaco_last_error().decode()


def _check(status: int, where: str):
    if status != TP_OK:
        raise TwoPaCoError(status, where, last_error())


@dataclass
class Genome:
    packed: np.ndarray
    n_bases: int
    n_runs: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.uint64))


def _genome_array(genomes):
    keep = []
    arr = (tp_genome * max(1, len(genomes)))()
    for i, g in enumerate(genomes):
        packed = np.ascontiguousarray(g.packed, dtype=np.uint8)
        runs = np.ascontiguousarray(g.n_runs, dtype=np.uint64).reshape(-1, 2)
        keep += [packed, runs]
        arr[i].packed = packed.ctypes.data if packed.size else None
        arr[i].n_bases = int(g.n_bases)
        arr[i].n_runs = runs.ctypes.data if runs.size else None
        arr[i].n_nruns = runs.shape[0]
    return arr, keep


@dataclass
class Result:
    """Host result: per-genome sorted junction positions, vertex ids (normalised
    k-mer, W words), strands and compacted edges."""
    junction_offset: np.ndarray
    junction_pos: np.ndarray
    vertex: np.ndarray          # (n_junctions, W) uint64, low word first
    strand: np.ndarray
    edges: np.ndarray           # EDGE_DTYPE
    stats: dict

    def junctions(self, g: int) -> np.ndarray:
        return self.junction_pos[self.junction_offset[g]:self.junction_offset[g + 1]]


def _stats_dict(st: tp_stats) -> dict:
    return {n: (float(getattr(st, n)) if t is ctypes.c_float else int(getattr(st, n)))
            for n, t in tp_stats._fields_}


class _ResultBlock:
    """Owns one library result block (header and arrays, page-locked); frees
    it when the last array viewing it is gone."""

    def __init__(self, addr: int):
        self.addr = addr

    def __del__(self):
        if self.addr and _lib is not None:
            _lib.twopaco_result_free(ctypes.c_void_p(self.addr))
        self.addr = 0


def _take_result(ptr: ctypes.c_void_p) -> Result:
    """Result arrays that view the library's block without copying it (a
    copy of a large result into fresh pages costs more than its transfer
    over the bus); the block goes back to the library's page-locked cache
    when the last of them is dropped."""
    r = tp_result.from_address(ptr.value)
    try:
        ng, nj, ne, W = r.n_genomes, r.n_junctions, r.n_edges, r.kmer_words
        stats = _stats_dict(r.stats)
        addrs = (r.junction_offset, r.junction_pos, r.vertex, r.strand, r.edges)
    except BaseException:
        lib().twopaco_result_free(ptr)
        raise
    owner = _ResultBlock(ptr.value)

    def arr(addr, n, dt):
        if n == 0:
            return np.zeros(0, dtype=dt)
        buf = (ctypes.c_uint8 * (n * np.dtype(dt).itemsize)).from_address(addr)
        buf._owner = owner  # the array's base keeps the block alive
        return np.ctypeslib.as_array(buf).view(dt)

    return Result(junction_offset=arr(addrs[0], ng + 1, np.uint64),
                  junction_pos=arr(addrs[1], nj, np.uint64),
                  vertex=arr(addrs[2], nj * W, np.uint64).reshape(nj, W),
                  strand=arr(addrs[3], nj, np.uint8),
                  edges=arr(addrs[4], ne, EDGE_DTYPE),
                  stats=stats)


def twopaco_build(genomes, k: int, bloom_bits: int, hash_count: int, flags: int = 0) -> Result:
    """Whole build from host genomes (``Genome`` records) to a host Result, on
    the current HIP device."""
    arr, keep = _genome_array(genomes)
    out = ctypes.c_void_p()
    _check(lib().twopaco_build_ex(ctypes.addressof(arr), len(genomes), k, bloom_bits,
                                  hash_count, flags, ctypes.byref(out)), "twopaco_build")
    return _take_result(out)


def bloom_bits_for(genomes, k: int, bits_per_edge: float = 16.0) -> int:
    """Power-of-two filter size at ``bits_per_edge`` bits per (k+1)-mer
    position of a genome set (tp_bloom_bits_for)."""
    arr, keep = _genome_array(genomes)
    b = int(lib().tp_bloom_bits_for(ctypes.addressof(arr), len(genomes), k, bits_per_edge))
    if b == 0:
        raise TwoPaCoError(TP_EINVAL, "bloom_bits_for", "invalid genomes or parameters")
    return b


def build_batch(sets, k: int, hash_count: int, flags: int = 0) -> list:
    """Whole build of independent genome sets ``[(genomes, bloom_bits), ...]``
    from host memory to one host Result per set (tp_build_batch)."""
    arr, keep = _set_array(list(sets))
    n = len(arr)
    outs = (ctypes.c_void_p * max(1, n))()
    _check(lib().tp_build_batch(ctypes.addressof(arr), n, k, hash_count, flags,
                                ctypes.addressof(outs)), "tp_build_batch")
    return [_take_result(ctypes.c_void_p(outs[i])) for i in range(n)]


def bench_random_access(buf, accesses: int, mode: int = 0, seed: int = 1, checksum=None,
                        stream=None) -> int:
    """Enqueue tp_bench_random_access on a torch device buffer (uint8);
    returns the exact number of accesses.  ``checksum``: an int64 device
    tensor of one element receiving the XOR of the loaded words."""
    done = ctypes.c_uint64()
    _check(lib().tp_bench_random_access(ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                        int(accesses), int(mode), int(seed),
                                        ctypes.c_void_p(checksum.data_ptr()),
                                        _stream_handle(stream), ctypes.byref(done)),
           "tp_bench_random_access")
    return int(done.value)


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _set_array(sets):
    """tp_set array for [(genomes, bloom_bits), ...]; returns it and the
    objects that must stay alive while it is in use."""
    arr = (tp_set * len(sets))()
    keep = []
    for i, (genomes, bloom_bits) in enumerate(sets):
        garr, gkeep = _genome_array(genomes)
        keep += [garr, gkeep]
        arr[i].genomes = ctypes.addressof(garr)
        arr[i].n_genomes = len(genomes)
        arr[i].reserved = 0
        arr[i].bloom_bits = int(bloom_bits)
    return arr, keep


class Plan:
    """Genome sets laid out for the device (tp_plan_* / tp_batch_*), reusable
    across runs.  ``Plan(genomes, k, b, h, flags)`` is a batch of one set;
    ``Plan.batch([(genomes, b), ...], k, h, flags)`` holds several sets, each
    with its own filter, table and results, run by the same launches."""

    def __init__(self, genomes, k: int, bloom_bits: int, hash_count: int, flags: int = 0,
                 _sets=None):
        self.sets = [(list(genomes), bloom_bits)] if _sets is None else \
            [(list(g), b) for g, b in _sets]
        self.genomes = [g for gs, _ in self.sets for g in gs]
        self.k, self.hash_count, self.flags = k, hash_count, flags
        self.bloom_bits = self.sets[0][1]
        h = ctypes.c_void_p()
        if _sets is None:
            arr, keep = _genome_array(self.genomes)
            _check(lib().tp_plan_create(ctypes.addressof(arr), len(self.genomes), k, bloom_bits,
                                        hash_count, flags, ctypes.byref(h)), "tp_plan_create")
        else:
            arr, keep = _set_array(self.sets)
            _check(lib().tp_batch_create(ctypes.addressof(arr), len(self.sets), k, hash_count,
                                         flags, ctypes.byref(h)), "tp_batch_create")
        self._h = h

    @classmethod
    def batch(cls, sets, k: int, hash_count: int, flags: int = 0) -> "Plan":
        """A plan over several genome sets: ``sets`` is [(genomes, bloom_bits), ...]."""
        return cls(None, k, None, hash_count, flags, _sets=list(sets))

    @property
    def handle(self):
        if not self._h:
            raise TwoPaCoError(TP_ESTATE, "Plan", "plan is closed")
        return self._h

    @property
    def input_bytes(self) -> int:
        return int(lib().tp_plan_input_bytes(self.handle))

    def genome_offset(self, g: int) -> int:
        return int(lib().tp_plan_genome_offset(self.handle, g))

    @property
    def bitmap_words(self) -> int:
        return int(lib().tp_plan_bitmap_words(self.handle))

    @property
    def n_strings(self) -> int:
        return int(lib().tp_plan_strings(self.handle))

    @property
    def n_sets(self) -> int:
        return int(lib().tp_plan_sets(self.handle))

    def set_first_genome(self, s: int) -> int:
        return int(lib().tp_plan_set_first_genome(self.handle, s))

    @property
    def rounds(self) -> int:
        """Algorithm 3's number of k-mer classes (tp_plan_set_rounds)."""
        return int(lib().tp_plan_rounds(self.handle))

    @rounds.setter
    def rounds(self, n: int) -> None:
        _check(lib().tp_plan_set_rounds(self.handle, int(n)), "tp_plan_set_rounds")

    def class_bounds(self, set_index: int = 0) -> np.ndarray:
        """Subrange bounds of the last run's classes (its rounds + 1 values)."""
        out = np.zeros(self.stats()["rounds"] + 1, dtype=np.uint32)
        _check(lib().tp_plan_class_bounds(self.handle, set_index, out.ctypes.data, out.size),
               "tp_plan_class_bounds")
        return out

    @property
    def config(self) -> dict:
        """Runtime knobs (tp_config): speed only, never results."""
        c = tp_config()
        _check(lib().tp_plan_get_config(self.handle, ctypes.byref(c)), "tp_plan_get_config")
        return {"wg_per_cu": list(c.wg_per_cu), "tile_order": int(c.tile_order),
                "table_load": float(c.table_load), "graphs": int(c.graphs),
                "pass2_slabs": int(c.pass2_slabs), "fill_dedup": int(c.fill_dedup),
                "table_shape": int(c.table_shape), "chunk_tiles": int(c.chunk_tiles),
                "fill_binned": int(c.fill_binned), "bin_chunk_tiles": int(c.bin_chunk_tiles),
                "bloom_bits_per_edge": int(c.bloom_bits_per_edge),
                "tile_queue": int(c.tile_queue), "record_binned": int(c.record_binned),
                "table_budget": int(c.table_budget), "record_passes": int(c.record_passes)}

    @config.setter
    def config(self, cfg: dict) -> None:
        cur = self.config
        cur.update(cfg)
        c = tp_config()
        for i, w in enumerate(cur["wg_per_cu"]):
            c.wg_per_cu[i] = int(w)
        c.tile_order = int(cur["tile_order"])
        c.table_load = float(cur["table_load"])
        c.graphs = int(cur.get("graphs", 0))
        c.pass2_slabs = int(cur.get("pass2_slabs", 2))
        c.fill_dedup = int(cur.get("fill_dedup", 1))
        c.table_shape = int(cur.get("table_shape", 0))
        c.chunk_tiles = int(cur.get("chunk_tiles", 1))
        c.fill_binned = int(cur.get("fill_binned", 0))
        c.bin_chunk_tiles = int(cur.get("bin_chunk_tiles", 0))
        c.bloom_bits_per_edge = int(cur.get("bloom_bits_per_edge", 0))
        c.tile_queue = int(cur.get("tile_queue", 0))
        c.record_binned = int(cur.get("record_binned", 0))
        c.table_budget = int(cur.get("table_budget", 0))
        c.record_passes = int(cur.get("record_passes", 0))
        _check(lib().tp_plan_set_config(self.handle, ctypes.byref(c)), "tp_plan_set_config")

    def autotune(self, d_input, cache_path=None, stream=None) -> dict:
        """Pick and apply the fastest knobs for this plan (tp_autotune)."""
        c = tp_config()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().tp_autotune(self.handle, ctypes.c_void_p(d_input.data_ptr()),
                                 _stream_handle(stream), path, ctypes.byref(c)), "tp_autotune")
        return self.config

    def upload(self, device=None, stream=None):
        """Allocate the device input (a torch uint8 tensor) and copy the genomes
        into it; returns the tensor."""
        import torch
        dev = torch.device("cuda") if device is None else torch.device(device)
        buf = torch.empty(max(16, self.input_bytes), dtype=torch.uint8, device=dev)
        arr, keep = _set_array(self.sets)
        _check(lib().tp_batch_upload(self.handle, ctypes.addressof(arr),
                                     ctypes.c_void_p(buf.data_ptr()), _stream_handle(stream)),
               "tp_batch_upload")
        torch.cuda.current_stream(dev).synchronize() if stream is None else stream.synchronize()
        return buf

    def upload_into(self, d_input, stream=None) -> None:
        """Copy the genomes into an existing device input (asynchronous on the
        stream; the genomes' host arrays must stay alive until it is done)."""
        arr, keep = _set_array(self.sets)
        _check(lib().tp_batch_upload(self.handle, ctypes.addressof(arr),
                                     ctypes.c_void_p(d_input.data_ptr()),
                                     _stream_handle(stream)), "tp_batch_upload")
        self._keep = keep

    def run(self, d_input, stream=None) -> None:
        _check(lib().tp_run(self.handle, ctypes.c_void_p(d_input.data_ptr()),
                            _stream_handle(stream)), "tp_run")

    def stats(self, set_index=None) -> dict:
        st = tp_stats()
        if set_index is None:
            _check(lib().tp_get_stats(self.handle, ctypes.byref(st)), "tp_get_stats")
        else:
            _check(lib().tp_get_set_stats(self.handle, set_index, ctypes.byref(st)),
                   "tp_get_set_stats")
        return _stats_dict(st)

    def device_outputs(self) -> dict:
        o = tp_device_outputs()
        _check(lib().tp_get_device_outputs(self.handle, ctypes.byref(o)), "tp_get_device_outputs")
        return {n: getattr(o, n) for n, _ in tp_device_outputs._fields_}

    def download(self, stream=None, set_index=None) -> Result:
        """Host copy of the last run's outputs: all genomes, or those of one set
        (genome indices relative to the set)."""
        out = ctypes.c_void_p()
        if set_index is None:
            _check(lib().tp_download(self.handle, _stream_handle(stream), ctypes.byref(out)),
                   "tp_download")
        else:
            _check(lib().tp_download_set(self.handle, set_index, _stream_handle(stream),
                                         ctypes.byref(out)), "tp_download_set")
        return _take_result(out)

    def set_bloom_bits(self, set_index: int = 0) -> int:
        """The set's filter size in bits (for a set created with bloom_bits 0,
        the size the plan chose at its current bloom_bits_per_edge)."""
        return int(lib().tp_plan_set_bloom_bits(self.handle, set_index))

    def debug_bloom(self, set_index: int = 0) -> np.ndarray:
        words = np.zeros(self.set_bloom_bits(set_index) // 32, dtype=np.uint32)
        _check(lib().tp_debug_set_bloom(self.handle, set_index, words.ctypes.data, words.size),
               "tp_debug_set_bloom")
        return words

    def debug_candidates(self) -> np.ndarray:
        words = np.zeros(self.bitmap_words, dtype=np.uint64)
        _check(lib().tp_debug_candidates(self.handle, words.ctypes.data, words.size),
               "tp_debug_candidates")
        return words

    def debug_table(self, set_index: int = 0):
        """(keys, masks) of the last run's exact table of one set: keys (n, W)
        uint64 normalised candidate k-mers, masks uint8 edge masks (bits 0-3
        in-bases, 4-7 out-bases), in slot order (tp_debug_table)."""
        n = ctypes.c_uint64()
        rc = lib().tp_debug_table(self.handle, set_index, None, None, 0, ctypes.byref(n))
        if rc not in (TP_OK, TP_EINVAL) or (rc == TP_EINVAL and n.value == 0):
            _check(rc, "tp_debug_table")
        W = 1 if self.k <= 31 else (2 if self.k <= 63 else 4)
        keys = np.zeros((max(1, n.value), W), dtype=np.uint64)
        masks = np.zeros(max(1, n.value), dtype=np.uint8)
        _check(lib().tp_debug_table(self.handle, set_index, keys.ctypes.data, masks.ctypes.data,
                                    keys.shape[0], ctypes.byref(n)), "tp_debug_table")
        return keys[:n.value], masks[:n.value]

    # ---- caller-owned memory (tp_run_ws)

    def workspace_layout(self, key_fraction: float = 1.0, junction_fraction: float = 1.0) -> dict:
        """Lay out a caller-owned workspace and output buffer for the given
        bounds (tp_plan_workspace_layout); returns the sizes and offsets."""
        L = tp_ws_layout()
        _check(lib().tp_plan_workspace_layout(self.handle, float(key_fraction),
                                              float(junction_fraction), ctypes.byref(L)),
               "tp_plan_workspace_layout")
        self._ws_layout = {n: int(getattr(L, n)) for n, _ in tp_ws_layout._fields_}
        return dict(self._ws_layout)

    def workspace_bytes(self) -> int:
        return int(lib().tp_plan_workspace_bytes(self.handle))

    def alloc_workspace(self, device=None):
        """(workspace, outputs) torch uint8 tensors of the current layout."""
        import torch
        L = self._ws_layout
        dev = torch.device("cuda") if device is None else torch.device(device)
        return (torch.empty(L["workspace_bytes"], dtype=torch.uint8, device=dev),
                torch.empty(L["output_bytes"], dtype=torch.uint8, device=dev))

    def prepare_workspace(self, workspace, stream=None) -> None:
        _check(lib().tp_plan_prepare_workspace(self.handle,
                                               ctypes.c_void_p(workspace.data_ptr()),
                                               _stream_handle(stream)),
               "tp_plan_prepare_workspace")

    def run_ws(self, d_input, workspace, outputs, stream=None) -> None:
        """Enqueue a whole run on caller memory (tp_run_ws); asynchronous."""
        _check(lib().tp_run_ws(self.handle, ctypes.c_void_p(d_input.data_ptr()),
                               ctypes.c_void_p(workspace.data_ptr()),
                               ctypes.c_void_p(outputs.data_ptr()), _stream_handle(stream)),
               "tp_run_ws")

    def run_noalloc(self, d_input, outputs, stream=None) -> None:
        """Enqueue a whole run on the library's fixed workspace (tp_run_noalloc):
        needs a current workspace layout of at most NOALLOC_WORKSPACE_MAX
        bytes; allocates nothing."""
        _check(lib().tp_run_noalloc(self.handle, ctypes.c_void_p(d_input.data_ptr()),
                                    ctypes.c_void_p(outputs.data_ptr()), _stream_handle(stream)),
               "tp_run_noalloc")

    def ws_views(self, outputs) -> dict:
        """Device views (torch tensors) of an output buffer: counts (16
        int64), joff, pos, vertex (n, W), strand, edges (n, 3) int64 words."""
        import torch
        L = self._ws_layout
        W = L["kmer_words"]
        mj, me = L["max_junctions"], L["max_edges"]
        ng = len(self.genomes)

        def sl(off, n, dt, width):
            return outputs[off:off + n * width].view(dt)

        return {"counts": sl(L["off_counts"], 16, torch.int64, 8),
                "joff": sl(L["off_joff"], ng + 1, torch.int64, 8),
                "pos": sl(L["off_pos"], mj, torch.int64, 8),
                "vertex": sl(L["off_vertex"], mj * W, torch.int64, 8).view(mj, W),
                "strand": outputs[L["off_strand"]:L["off_strand"] + mj],
                "edges": sl(L["off_edges"], me * 3, torch.int64, 8).view(me, 3)}

    def ws_counts(self, outputs) -> dict:
        """Counts and status of the run that wrote an output buffer (reads it
        back: the caller synchronises first)."""
        c = self.ws_views(outputs)["counts"].cpu().numpy().view(np.uint64)
        return {n: int(c[i]) for i, n in enumerate(WS_COUNT_FIELDS)}

    def ws_result(self, outputs) -> Result:
        """Host Result from an output buffer (its counts must show a complete run)."""
        v = self.ws_views(outputs)
        cnt = self.ws_counts(outputs)
        nj, ne = cnt["junctions"], cnt["edges"]
        ed = v["edges"][:ne].cpu().numpy().view(np.uint64)
        edges = np.zeros(ne, dtype=EDGE_DTYPE)
        if ne:
            edges["genome"] = (ed[:, 0] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
            edges["from_pos"] = ed[:, 1]
            edges["to_pos"] = ed[:, 2]
        return Result(junction_offset=v["joff"].cpu().numpy().view(np.uint64),
                      junction_pos=v["pos"][:nj].cpu().numpy().view(np.uint64),
                      vertex=v["vertex"][:nj].cpu().numpy().view(np.uint64),
                      strand=v["strand"][:nj].cpu().numpy(),
                      edges=edges, stats=cnt)

    def bitmap_positions(self, words: np.ndarray) -> list:
        """Split a position bitmap into per-genome sorted positions (all
        genomes of the plan, in order)."""
        bits = np.unpackbits(words.view(np.uint8), bitorder="little")
        out = []
        for g, gen in enumerate(self.genomes):
            base = self.genome_offset(g) * 4
            out.append(np.flatnonzero(bits[base:base + int(gen.n_bases)]).astype(np.uint64))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().tp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (tp_server_*): jobs submitted at any time, admitted by an
    HBM budget, small compatible jobs batched into one plan, workers on
    their own streams.  ``submit`` copies the genomes; ``wait`` returns the
    job's Result and its times."""

    def __init__(self, hbm_budget: int, workers: int = 2, max_batch: int = 32,
                 batch_max_bases: int = 20_000_000, batch_total_bases: int = 400_000_000,
                 wg_per_cu: int = 0, express_workers: int = 0, express_cus: int = 0,
                 table_budget_mib: int = 0):
        o = tp_server_opts(hbm_budget=int(hbm_budget), workers=workers, max_batch=max_batch,
                           batch_max_bases=int(batch_max_bases),
                           batch_total_bases=int(batch_total_bases), wg_per_cu=wg_per_cu,
                           express_workers=express_workers, express_cus=express_cus,
                           table_budget_mib=int(table_budget_mib))
        h = ctypes.c_void_p()
        _check(lib().tp_server_create(ctypes.byref(o), ctypes.byref(h)), "tp_server_create")
        self._h = h

    @property
    def handle(self):
        if not self._h:
            raise TwoPaCoError(TP_ESTATE, "Server", "server is closed")
        return self._h

    def submit(self, genomes, k: int, bloom_bits: int, hash_count: int, flags: int = 0) -> int:
        arr, keep = _genome_array(genomes)
        jid = ctypes.c_uint64()
        _check(lib().tp_server_submit(self.handle, ctypes.addressof(arr), len(genomes), k,
                                      bloom_bits, hash_count, flags, ctypes.byref(jid)),
               "tp_server_submit")
        return int(jid.value)

    def wait(self, job_id: int, timeout_ms: int = -1, keep: bool = True):
        """(Result, info) of a finished job; with keep=False the result is
        freed unread and (None, info) returned."""
        out = ctypes.c_void_p()
        info = tp_job_info()
        _check(lib().tp_server_wait(self.handle, job_id, timeout_ms, ctypes.byref(out),
                                    ctypes.byref(info)), "tp_server_wait")
        meta = {n: getattr(info, n) for n, _ in tp_job_info._fields_}
        if not keep:
            lib().twopaco_result_free(out)
            return None, meta
        return _take_result(out), meta

    def poll(self, job_id: int, keep: bool = True):
        """(Result, info) of a finished job, or None while it is queued or
        running (tp_server_poll)."""
        out = ctypes.c_void_p()
        info = tp_job_info()
        rc = lib().tp_server_poll(self.handle, job_id, ctypes.byref(out), ctypes.byref(info))
        if rc == TP_EPENDING:
            return None
        _check(rc, "tp_server_poll")
        meta = {n: getattr(info, n) for n, _ in tp_job_info._fields_}
        if not keep:
            lib().twopaco_result_free(out)
            return None, meta
        return _take_result(out), meta

    def stats(self) -> dict:
        st = tp_server_stats()
        _check(lib().tp_server_get_stats(self.handle, ctypes.byref(st)), "tp_server_get_stats")
        return {n: int(getattr(st, n)) for n, _ in tp_server_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().tp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
