"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, validates arguments and lays genomes out
as documented.  No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1602_05856_amd as tp
import synth
from helpers import to_genomes

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "twopaco.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(?:int|void|uint32_t|uint64_t|const char \*)\s*\*?\s*(\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = tp.lib()
    names = declared_functions()
    assert len(names) >= 24
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(tp.SIGNATURES), "binding signatures out of sync with the header"


def _plan_status(genomes, k=25, b=2**20, h=3, flags=0):
    arr, keep = tp._genome_array(genomes)
    h_ = ctypes.c_void_p()
    rc = tp.lib().tp_plan_create(ctypes.addressof(arr), len(genomes), k, b, h, flags,
                                 ctypes.byref(h_))
    if rc == 0:
        tp.lib().tp_plan_destroy(h_)
    else:
        assert not h_.value
        assert tp.last_error()
    return rc


def test_parameter_validation():
    g = to_genomes([np.zeros(100, np.uint8)])
    assert _plan_status(g) == tp.TP_OK
    for k in (0, 128, 200):
        assert _plan_status(g, k=k) == tp.TP_EINVAL
    for b in (16, 33, 2**20 + 1, 2**41):
        assert _plan_status(g, b=b) == tp.TP_EINVAL
    for h in (0, 17):
        assert _plan_status(g, h=h) == tp.TP_EINVAL
    assert _plan_status(g, flags=8) == tp.TP_EINVAL
    assert _plan_status(g, b=32, flags=tp.TP_FLAG_BLOCKED_FILTER) == tp.TP_EINVAL
    assert _plan_status(g, b=64, flags=tp.TP_FLAG_BLOCKED_FILTER) == tp.TP_OK
    assert _plan_status(g, k=1, b=32, h=1) == tp.TP_OK
    assert _plan_status(g, k=63, b=2**40, h=16) == tp.TP_OK
    assert _plan_status(g, k=64) == tp.TP_OK and _plan_status(g, k=127) == tp.TP_OK


@pytest.mark.parametrize("runs", [
    [(10, 5), (12, 3)],       # overlapping
    [(20, 5), (10, 5)],       # unsorted
    [(10, 0)],                # empty
    [(95, 10)],               # past the end
    [(100, 1)],               # starts at the end
])
def test_bad_n_runs(runs):
    g = tp.Genome(packed=np.zeros(25, np.uint8), n_bases=100,
                  n_runs=np.array(runs, dtype=np.uint64))
    assert _plan_status([g]) == tp.TP_EINVAL


def test_layout_and_strings():
    codes = synth.random_genomes(3, 6, 0, 3000, n_frac=0.0)
    codes[2][100:400] = 4
    codes[4][:50] = 4
    gs = to_genomes(codes)
    k = 25
    p = tp.Plan(gs, k, 2**16, 2)
    offs = [p.genome_offset(i) for i in range(len(gs))]
    assert offs[0] == 0
    for i in range(1, len(gs)):
        assert offs[i] % 64 == 0
        assert offs[i] >= offs[i - 1] + (gs[i - 1].n_bases + 3) // 4
    assert p.input_bytes >= offs[-1] + (gs[-1].n_bases + 3) // 4 + 24
    assert p.bitmap_words * 64 >= offs[-1] * 4 + gs[-1].n_bases
    # strings: maximal N-free runs of length >= k
    want = 0
    for c in codes:
        run = 0
        for x in list(c) + [4]:
            if x > 3:
                want += run >= k
                run = 0
            else:
                run += 1
    assert p.n_strings == want
    p.close()


def test_outputs_before_run_are_refused():
    p = tp.Plan(to_genomes([np.zeros(100, np.uint8)]), 5, 2**10, 2)
    with pytest.raises(tp.TwoPaCoError) as e:
        p.stats()
    assert e.value.status == tp.TP_ESTATE
    with pytest.raises(tp.TwoPaCoError):
        p.debug_bloom()
    p.close()


def _batch_status(sets, k=25, h=3, flags=0):
    arr, keep = tp._set_array(sets)
    h_ = ctypes.c_void_p()
    rc = tp.lib().tp_batch_create(ctypes.addressof(arr) if sets else None, len(sets), k, h,
                                  flags, ctypes.byref(h_))
    if rc == 0:
        tp.lib().tp_plan_destroy(h_)
    else:
        assert not h_.value
        assert tp.last_error()
    return rc


def test_batch_validation():
    g = to_genomes([np.zeros(100, np.uint8)])
    assert _batch_status([(g, 2**10)]) == tp.TP_OK
    assert _batch_status([]) == tp.TP_EINVAL
    assert _batch_status([(g, 2**10), ([], 2**12), (g, 2**20)]) == tp.TP_OK
    assert _batch_status([(g, 2**10), (g, 1000)]) == tp.TP_EINVAL
    assert "set 1" in tp.last_error()
    assert _batch_status([(g, 2**10), (g, 32)], flags=tp.TP_FLAG_BLOCKED_FILTER) == tp.TP_EINVAL
    assert _batch_status([(g, 64)], flags=tp.TP_FLAG_BLOCKED_FILTER) == tp.TP_OK
    assert _batch_status([(g, 2**10)], k=128) == tp.TP_EINVAL
    bad = tp.Genome(packed=np.zeros(25, np.uint8), n_bases=100,
                    n_runs=np.array([(20, 5), (10, 5)], dtype=np.uint64))
    assert _batch_status([(g, 2**10), ([bad], 2**10)]) == tp.TP_EINVAL
    assert "set 1" in tp.last_error()


def test_batch_layout():
    codes = [synth.random_genomes(40 + s, 1 + s % 3, 0, 5000) for s in range(5)]
    sets = [(to_genomes(c), 2**(10 + s)) for s, c in enumerate(codes)]
    k = 21
    p = tp.Plan.batch(sets, k, 3)
    assert p.n_sets == 5
    first = 0
    for s, (gs, b) in enumerate(sets):
        assert p.set_first_genome(s) == first
        first += len(gs)
    # set filters are disjoint, in order, 256-byte aligned
    offs = [int(tp.lib().tp_plan_set_bloom_offset(p.handle, s)) for s in range(5)]
    assert offs[0] == 0
    for s in range(1, 5):
        assert offs[s] % 64 == 0 and offs[s] >= offs[s - 1] + sets[s - 1][1] // 32
    assert int(tp.lib().tp_plan_bloom_words(p.handle)) >= offs[-1] + sets[-1][1] // 32
    # genomes of all sets in one input, in order
    allg = [g for gs, _ in sets for g in gs]
    goffs = [p.genome_offset(i) for i in range(len(allg))]
    for i in range(1, len(allg)):
        assert goffs[i] % 512 == 0 and goffs[i] >= goffs[i - 1] + (allg[i - 1].n_bases + 3) // 4
    assert p.n_strings == sum(1 for g in allg if g.n_bases >= k)
    p.close()


def test_auto_sized_filters():
    """A set given bloom_bits 0 gets the filter tp_bloom_bits_for gives at
    the plan's bits per (k+1)-mer (16 by default); changing the density re-lays
    out the filter pool, beside sets of fixed size."""
    codes = [synth.random_genomes(60 + s, 1 + s % 3, 1000, 40_000, n_frac=0.01)
             for s in range(4)]
    fixed = 2**14
    sets = [(to_genomes(c), 0 if s % 2 == 0 else fixed) for s, c in enumerate(codes)]
    k = 25
    p = tp.Plan.batch(sets, k, 3)
    for bpe in (0, 8, 32, 3, 16):
        if bpe:
            p.config = {"bloom_bits_per_edge": bpe}
        for s, (gs, b) in enumerate(sets):
            want = tp.bloom_bits_for(gs, k, bpe or 16) if b == 0 else fixed
            assert p.set_bloom_bits(s) == want, (bpe, s)
        offs = [int(tp.lib().tp_plan_set_bloom_offset(p.handle, s)) for s in range(4)]
        assert offs[0] == 0
        for s in range(1, 4):
            assert offs[s] % 64 == 0 and offs[s] >= offs[s - 1] + p.set_bloom_bits(s - 1) // 32
        assert int(tp.lib().tp_plan_bloom_words(p.handle)) >= offs[-1] + p.set_bloom_bits(3) // 32
    p.close()
    one = tp.Plan(sets[0][0], k, 0, 3)
    assert one.set_bloom_bits(0) == tp.bloom_bits_for(sets[0][0], k)
    one.close()


def test_bloom_bits_for():
    def want(lengths_and_runs, k, bpe):
        edges = 0
        for n, runs in lengths_and_runs:
            cuts = [0]
            for s, l in runs:
                cuts += [s, s + l]
            cuts.append(n)
            for a, z in zip(cuts[::2], cuts[1::2]):
                edges += max(0, z - a - k)
        b = 64
        while b < bpe * edges:
            b *= 2
        return b

    cases = [[(100, [])], [(31, [])], [(32, [])], [(10_000, [(100, 50), (5000, 1)])],
             [(5000, []), (7000, [(0, 10)]), (0, [])], [(1 << 20, [])]]
    for case in cases:
        gs = [tp.Genome(packed=np.zeros((n + 3) // 4, np.uint8), n_bases=n,
                        n_runs=np.array(r, dtype=np.uint64).reshape(-1, 2)) for n, r in case]
        for k, bpe in ((31, 16.0), (25, 16.0), (5, 3.5)):
            assert tp.bloom_bits_for(gs, k, bpe) == want(case, k, bpe), (case, k, bpe)
    assert tp.bloom_bits_for([tp.Genome(np.zeros(25, np.uint8), 100)], 31) == 2048  # 69 edges
    with pytest.raises(tp.TwoPaCoError):
        tp.bloom_bits_for([tp.Genome(np.zeros(25, np.uint8), 100)], 31, 0.0)


def test_config_defaults_and_validation():
    g = to_genomes([np.zeros(3000, np.uint8)])
    p = tp.Plan(g, 25, 2**16, 3)
    c = p.config
    assert c == {"wg_per_cu": [0, 0, 6, 6], "tile_order": 0, "table_load": pytest.approx(0.7),
                 "graphs": 0, "pass2_slabs": 2, "fill_dedup": 1, "table_shape": 0,
                 "chunk_tiles": 1, "fill_binned": 0, "bin_chunk_tiles": 0,
                 "bloom_bits_per_edge": 0, "tile_queue": 1, "record_binned": 0,
                 "table_budget": 0, "record_passes": 0}
    p.config = {"chunk_tiles": 64, "table_budget": 1 << 40}
    p.config = {"record_binned": 2, "record_passes": 64}
    assert p.config["record_binned"] == 2 and p.config["record_passes"] == 64
    assert p.config["chunk_tiles"] == 64 and p.config["table_budget"] == 1 << 40
    p.config = {"fill_binned": 2, "bin_chunk_tiles": 1 << 20}
    assert p.config["fill_binned"] == 2 and p.config["bin_chunk_tiles"] == 1 << 20
    p.config = {"wg_per_cu": [1, 2, 3, 4], "tile_order": 1, "table_load": 2.0}
    assert p.config["wg_per_cu"] == [1, 2, 3, 4] and p.config["tile_order"] == 1
    for bad in ({"wg_per_cu": [65, 0, 0, 0]}, {"tile_order": 2}, {"table_load": 0.01},
                {"table_load": 17.0}, {"table_load": float("nan")}, {"graphs": 2},
                {"pass2_slabs": 8}, {"fill_dedup": 2}, {"table_shape": 3},
                {"chunk_tiles": 0}, {"chunk_tiles": 65}, {"fill_binned": 3},
                {"bin_chunk_tiles": (1 << 20) + 1}, {"bloom_bits_per_edge": 257},
                {"tile_queue": 2}, {"record_binned": 3}, {"record_passes": 65}):
        with pytest.raises(tp.TwoPaCoError) as e:
            p.config = bad
        assert e.value.status == tp.TP_EINVAL
    assert p.config["wg_per_cu"] == [1, 2, 3, 4]  # unchanged by a refused config
    p.close()
    b = tp.Plan.batch([(g, 2**12), (g, 2**12)], 25, 3)
    assert b.config["table_load"] == pytest.approx(0.5)
    b.close()


def test_server_option_validation():
    # refused before any device call, so these run without a GPU
    for kw in ({"workers": 0}, {"workers": 17}, {"max_batch": 0}, {"hbm_budget": 0},
               {"express_workers": 2}, {"workers": 1, "express_workers": 1},
               {"express_cus": 8}):
        args = dict(hbm_budget=1 << 30, workers=2, max_batch=4)
        args.update(kw)
        with pytest.raises(tp.TwoPaCoError) as e:
            tp.Server(**args)
        assert e.value.status == tp.TP_EINVAL


def test_rounds_validation():
    p = tp.Plan(to_genomes([np.zeros(3000, np.uint8)]), 25, 2**16, 3)
    assert p.rounds == 1
    for bad in (0, 65):
        with pytest.raises(tp.TwoPaCoError) as e:
            p.rounds = bad
        assert e.value.status == tp.TP_EINVAL
    p.rounds = 64
    assert p.rounds == 64
    with pytest.raises(tp.TwoPaCoError) as e:
        p.class_bounds()
    assert e.value.status == tp.TP_ESTATE
    p.close()


def test_one_hip_runtime_whatever_the_import_order():
    # loading the library before torch must not leave two HIP runtimes in the
    # process (they would not share the device)
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import paper_1602_05856_amd as tp\n"
            "tp.lib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n" % root)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "1"


def test_workspace_layout_host_only():
    codes = synth.random_genomes(11, 5, 500, 20000, n_frac=0.001)
    gs = to_genomes(codes)
    for k, flags, rounds in ((25, 0, 1), (40, tp.TP_FLAG_BLOCKED_FILTER, 3), (100, 0, 1),
                             (31, tp.TP_FLAG_PASS1_ONLY, 2)):
        p = tp.Plan(gs, k, 2**16, 3, flags)
        p.rounds = rounds
        assert p.workspace_bytes() == 0  # no layout yet
        small = p.workspace_layout(0.1, 0.2)
        big = p.workspace_layout(1.0, 1.0)
        assert p.workspace_bytes() == big["workspace_bytes"]
        W = 1 if k <= 31 else (2 if k <= 63 else 4)
        assert big["kmer_words"] == W and big["rounds"] == rounds
        if flags & tp.TP_FLAG_PASS1_ONLY:
            assert big["table_slots"] == 0
        else:
            assert big["table_slots"] > small["table_slots"] > 0
            assert big["workspace_bytes"] > small["workspace_bytes"]
        positions = sum(max(0, len(s) - k + 1) for c in codes
                        for s in "".join("N" if x > 3 else "A" for x in c).split("N"))
        assert big["max_junctions"] == positions
        assert small["max_junctions"] < big["max_junctions"]
        # output regions: in order, 256-byte aligned, inside the buffer
        offs = [big[n] for n in ("off_counts", "off_joff", "off_pos", "off_vertex",
                                 "off_strand", "off_edges")]
        assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
        assert big["off_joff"] - big["off_counts"] >= 128
        assert big["off_vertex"] - big["off_pos"] >= 8 * big["max_junctions"]
        assert big["output_bytes"] >= big["off_edges"] + 24 * big["max_edges"]
        for n in ("ws_off_candidates", "ws_off_junction_bits", "ws_off_bloom",
                  "ws_off_set_counters"):
            assert big[n] % 256 == 0 and big[n] < big["workspace_bytes"]
        # a run needs the workspace prepared for the current layout (checked
        # before any device call)
        rc = tp.lib().tp_run_ws(p.handle, ctypes.c_void_p(256), ctypes.c_void_p(512),
                                ctypes.c_void_p(1024), None)
        assert rc == tp.TP_ESTATE and "prepared" in tp.last_error()
        # changing rounds or knobs invalidates the layout
        p.rounds = rounds
        assert p.workspace_bytes() == 0
        p.workspace_layout(1.0, 1.0)
        p.config = {"table_load": 0.5}
        assert p.workspace_bytes() == 0
        for kf, jf in ((0, 1), (1.5, 1), (1, 0), (1, 2)):
            with pytest.raises(tp.TwoPaCoError) as e:
                p.workspace_layout(kf, jf)
            assert e.value.status == tp.TP_EINVAL
        p.close()


def test_debug_table_and_build_batch_validation():
    p = tp.Plan(to_genomes([np.zeros(100, np.uint8)]), 5, 2**10, 2)
    n = ctypes.c_uint64()
    assert tp.lib().tp_debug_table(p.handle, 0, None, None, 0, ctypes.byref(n)) == tp.TP_ESTATE
    assert tp.lib().tp_debug_table(p.handle, 3, None, None, 0, ctypes.byref(n)) == tp.TP_EINVAL
    p.close()
    outs = (ctypes.c_void_p * 1)()
    assert tp.lib().tp_build_batch(None, 0, 25, 3, 0, ctypes.addressof(outs)) == tp.TP_EINVAL
    assert tp.lib().tp_build_batch(None, 0, 25, 3, 0, None) == tp.TP_EINVAL
