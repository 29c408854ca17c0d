#!/usr/bin/env python3
"""Junction-finding throughput on one MI355X.

Headline workload: 8 primate-scale genomes of 3 Gbp each (~24 Gbp) from one
random base, 1-8% pairwise divergence with indels, interspersed repeat
families and runs of N; k = 25, Bloom filter 2^36 bits (8 GiB, in HBM),
h = 5, the blocked filter layout, one round.  Synthetic stand-in for the
8-primate benchmark of the paper's Results section: the largest workload
that one GPU holds, and the one whose filter and exact table live in HBM.

A step is one pass of the whole device path over the resident packed input:
sentinels, Bloom fill, Bloom query (candidates), exact-table record,
junction decision, ordered compaction and compacted edges.  The metric is
input gigabases per second (non-N bases / step time).  Secondary legs (each
switchable): the standard filter layout on the same input; the 62 x 5 Mbp
bacterial workload (k = 25, 63, 100); the batched form (256 sets) against
one set per launch and as one captured graph; the serving loop against one
set per launch on the same request mix; the random-access rate of the
memory system by footprint; the CPU oracle on a stated prefix.  Prints one
JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
MALL_BYTES = 256 << 20  # last-level cache: a structure this small is probed on chip
GRANULE = 64            # bytes the memory system moves per random word access: every
                        # L2-to-fabric read request of these kernels is 64 B or more
                        # (rocprofv3 TCC_EA0_RDREQ_32B_sum = 0), so no access costs less
PROFILES = os.path.join(ROOT, "profiles")
KERNELS = ("fill", "query", "record", "decide", "compact")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def genomes_for(codes):
    import paper_1602_05856_amd as tp
    import synth
    out = []
    for c in codes:
        packed, runs = synth.pack(c)
        out.append(tp.Genome(packed=packed, n_bases=int(c.size), n_runs=runs))
    return out


def table_arrays(k, W):
    """Table arrays one insert or lookup touches: 1 (key and mask in one
    word), 2 (key word + mask byte), or the key words of a wide key (top
    word, low word, middle words) plus a mask byte unless the mask fits in
    the top word."""
    if k <= 27:
        return 1
    if W == 1:
        return 2
    himask = 2 * k <= 64 * (W - 1) + 54
    return (2 if W == 2 else 3) + (0 if himask else 1)


def slot_bytes(k, W):
    return 8 * W + (0 if k <= 27 or (W >= 2 and 2 * k <= 64 * (W - 1) + 54) else 1)


def algorithmic_bytes(c, bases, k, W, h, blocked, filter_bytes, table_bytes, nonzero_granules):
    """Bytes each kernel must move to or from HBM under the direct-probe model,
    from the method's own counts (not kernel counters):
      genome     the packed input streamed once per kernel, 2 bits per base;
      bitmaps    candidate and junction bitmaps at one bit per position;
      outputs    junctions and edges as written;
      probes     one GRANULE per random filter or table access the method
                 makes -- fill: one per (k+1)-mer (blocked) or h (standard),
                 plus every filter granule left non-zero written once;
                 query: one filter block per position (blocked); standard:
                 six membership tests per position, each testing bits until
                 the first clear one, (1 - r^h) / (1 - r) words on average
                 for a filter whose fraction r of bits is set (the fill
                 ratio of the Theoretical Analysis); record and
                 decision: the table arrays of one slot per candidate --
                 charged only for a structure larger than the 256 MB
                 last-level cache (a smaller one is probed on chip).
    c: positions, edge_positions, candidates, junctions, edges, bloom_popcount."""
    pos, epos, cand = c["positions"], c["edge_positions"], c["candidates"]
    nj, ne = c["junctions"], c["edges"]
    genome = bases / 4
    f_hbm = filter_bytes > MALL_BYTES
    t_hbm = table_bytes > MALL_BYTES
    arrays = table_arrays(k, W)
    fill_probes = epos * (1 if blocked else h)
    if blocked:
        query_probes = pos
    else:
        r = min(c["bloom_popcount"] / (filter_bytes * 8), 1 - 1e-12)
        query_probes = pos * 6 * (1 - r ** h) / (1 - r)
    out = {
        "fill": genome + (GRANULE * (fill_probes + nonzero_granules) if f_hbm else 0),
        "query": genome + pos / 8 + (GRANULE * query_probes if f_hbm and query_probes else 0),
        "record": genome + pos / 8 + (GRANULE * arrays * cand if t_hbm else 0),
        "decide": genome + 2 * pos / 8 + (GRANULE * arrays * cand if t_hbm else 0),
        "compact": pos / 8 + genome + nj * (8 + 8 * W + 1) + ne * 24,
    }
    probes = {"fill": fill_probes, "query": query_probes, "record": arrays * cand,
              "decide": arrays * cand}
    return out, probes, {"filter_in_hbm": f_hbm, "table_in_hbm": t_hbm}


def binned_fill_bytes(st, c, bases, filter_bytes, fill_ms):
    """Streaming bytes of the binned fill (one round): the input read once;
    one 8-byte slot per position staged and read back; every item (one per
    edge position) written by the bucket scatter, read twice and written by
    the region split, read by the apply; the filter written by the first
    chunk and read and written by every later one.  These replace the
    direct-probe bytes in the fill's roofline entry when the fill ran
    binned (the model follows the schedule)."""
    chunks = st["fill_chunks"]
    items = c["edge_positions"]
    nbytes = (bases / 4 + 16 * c["positions"] + 8 * items * (1 + 3 + 1) +
              filter_bytes * (2 * chunks - 1))
    gbs = nbytes / (fill_ms * 1e-3) / 1e9
    return {"chunks": chunks, "streaming_bytes": nbytes, "achieved_gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS}


def binned_record_bytes(st, c, bases, table_bytes, record_ms):
    """Streaming bytes of the binned record (one round): every pass reads
    the input and the candidate bitmap; every item (one per candidate) is
    staged, read by the histogram and the bucket scatter, written by it,
    read twice and written by the block split and read by the apply (8 bytes
    each time); the table is written once, block by block.  These replace
    the direct-probe bytes in the record's roofline entry when the record
    ran binned."""
    passes = st["record_passes"]
    nbytes = (passes * (bases / 4 + c["positions"] / 8) + 64 * c["candidates"] + table_bytes)
    gbs = nbytes / (record_ms * 1e-3) / 1e9
    return {"passes": passes, "streaming_bytes": nbytes, "achieved_gbs": gbs,
            "frac": gbs / HBM_PEAK_GBS}


def nonzero_granules_dev(ptr, n_words):
    """Filter granules (GRANULE bytes) with any bit set, counted on the device
    from the filter words (uint32) at a device pointer."""
    import torch
    t = dev_view(ptr, n_words, "<i4")
    per = GRANULE // 4
    total = 0
    chunk = per << 24
    for i in range(0, n_words, chunk):
        blk = t[i:i + chunk].view(-1, per)
        total += int((blk != 0).any(dim=1).sum())
    torch.cuda.synchronize()
    return total


class _DevArray:
    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 3}


def dev_view(ptr, n, typestr):
    import torch
    return torch.as_tensor(_DevArray(ptr, n, typestr), device="cuda")


# The sources that define the pipeline's kernels and their launches (grids,
# tile walks, buffer sizing): counters taken on other sources no longer
# describe these kernels.  The serving loop, the tuner, the caller-memory and
# no-allocation entry points and the memory benchmark only call them.
KERNEL_SOURCES = ("compact.hip", "device.hpp", "layout.hpp", "pass1.hip", "pass2.hip",
                  "runtime.cpp", "runtime.hpp")


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1602_05856_amd", "csrc")
    for name in KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(tag, kernel):
    """HBM bytes per run of phase `kernel` from the committed rocprofv3 counter
    summary of workload `tag`, if it was taken on the current kernel sources;
    else (None, None)."""
    path = os.path.join(PROFILES, "traffic_%s.txt" % tag)
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest():
        return None, None
    kr = rec.get("kernels", {}).get(kernel, {})
    return kr.get("bytes_per_run"), kr.get("raw_bytes_per_run")


def roofline(alg, kernel_ms, tag):
    dom = max(("fill", "query", "record", "decide"), key=lambda n: kernel_ms[n])
    achieved = alg[dom] / (kernel_ms[dom] * 1e-3) / 1e9
    traffic, traffic_raw = measured_traffic(tag, dom)
    p12 = sum(alg[n] for n in ("fill", "query", "record", "decide"))
    t12 = sum(kernel_ms[n] for n in ("fill", "query", "record", "decide")) * 1e-3
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unscaled": traffic_raw, "algorithmic_bytes": alg[dom], "granule": GRANULE,
            "pipeline_frac": p12 / t12 / 1e9 / HBM_PEAK_GBS,
            "per_kernel_frac": {n: alg[n] / (kernel_ms[n] * 1e-3) / 1e9 / HBM_PEAK_GBS
                                for n in kernel_ms}}


def tune(plan, d_input, args):
    if args.config:
        plan.config = json.loads(args.config)
        return plan.config
    if not args.tune:
        return plan.config
    t0 = time.perf_counter()
    cfg = plan.autotune(d_input, args.tune_cache)
    log("autotuned in %.1fs: %s" % (time.perf_counter() - t0, cfg))
    return cfg


def run_steps(plan, d_input, steps, warmup, stream):
    import torch
    for i in range(warmup):
        plan.run(d_input, stream)
        log("warmup %d: %.2f ms" % (i, plan.stats()["ms_total"]))
    torch.cuda.synchronize()
    per_step = []
    t0 = time.perf_counter()
    for i in range(steps):
        plan.run(d_input, stream)
        per_step.append(plan.stats())
        if steps > 4:
            log("step %d: %.2f ms" % (i, per_step[-1]["ms_total"]))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / max(1, steps), per_step


def kernel_avg(per):
    return {n: sum(s["ms_" + n] for s in per) / len(per) for n in KERNELS}


def counts_of(st):
    return {n: st[n] for n in ("positions", "edge_positions", "candidates", "junctions",
                               "edges", "table_keys", "table_capacity", "query_probes",
                               "fill_atomics", "table_probes", "bloom_popcount")}


# ------------------------------------------------------------------ primate

PRIMATE_K, PRIMATE_B_LOG2, PRIMATE_H = 25, 36, 5


def primate_input():
    import paper_1602_05856_amd as tp
    import synth
    t0 = time.perf_counter()
    gs = synth.primate(0, 1.0, packed=True)
    bases = sum(int(m) - int(r[:, 1].sum()) for _, m, r in gs)
    genomes = [tp.Genome(packed=p, n_bases=m, n_runs=r) for p, m, r in gs]
    log("primate workload: %d genomes, %.2f Gbp (%.2f Gbp without N) in %.1fs" % (
        len(gs), sum(m for _, m, _ in gs) / 1e9, bases / 1e9, time.perf_counter() - t0))
    return gs, genomes, bases


def primate_leg(args, stream, genomes, bases, flags, steps, warmup, d_in=None, order=None):
    """Time the primate workload: one round, the table at the configured load
    target (an any-size table of ~1.1e10 slots when blocked), and the
    faster of the two pass-2 tile orders, picked on the first two warmup
    runs (homologous tiles of 3 Gbp genomes drift apart through indels)
    unless given."""
    import torch

    import paper_1602_05856_amd as tp
    k, b, h = PRIMATE_K, 1 << PRIMATE_B_LOG2, PRIMATE_H
    W = 1
    blocked = bool(flags & tp.TP_FLAG_BLOCKED_FILTER)
    plan = tp.Plan(genomes, k, b, h, flags)
    if d_in is None:
        d_in = plan.upload()
    plan.rounds = args.primate_rounds
    plan.config = {"table_load": args.primate_load}
    t = {}
    for ps in ((2, 0) if order is None and warmup >= 2 else ()):
        plan.config = {"pass2_slabs": ps}
        plan.run(d_in, stream)
        st = plan.stats()
        t[ps] = st["ms_record"] + st["ms_decide"]
        log("primate %s warmup (pass2 order %d): %.1f ms" % (
            "blocked" if blocked else "standard", ps, st["ms_total"]))
    if order is None:
        order = min(t, key=t.get) if t else 2
    plan.config = {"pass2_slabs": order}
    ms, per = run_steps(plan, d_in, steps, max(0, warmup - len(t)), stream)
    st = dict(per[-1])
    km = kernel_avg(per)
    out = plan.device_outputs()
    nz = nonzero_granules_dev(out["bloom"], b // 32)
    c = counts_of(st)
    alg, probes, where = algorithmic_bytes(c, bases, k, W, h, blocked, b // 8,
                                           c["table_capacity"] * slot_bytes(k, W), nz)
    rec = {"value": bases / 1e9 / (ms * 1e-3), "ms_per_step": ms, "steps": steps,
           "config": plan.config, "kernel_ms": km,
           "pass12_ms": sum(km[n] for n in ("fill", "query", "record", "decide")),
           "counts": c, "nonzero_filter_granules": nz, "algorithmic_bytes": alg,
           "method_probes": probes, "residency": where,
           "roofline": roofline(alg, km, "primate_k25_%s" % ("blocked" if blocked else
                                                             "standard"))}
    if st["fill_chunks"] or st["record_passes"]:
        # the fill or the record ran binned: its bytes are that schedule's
        # (streaming), the direct-probe figure is kept beside them
        if st["fill_chunks"]:
            rec["binned_fill"] = binned_fill_bytes(st, c, bases, b // 8, km["fill"])
            rec["binned_fill"]["direct_probe_bytes"] = alg["fill"]
            alg["fill"] = rec["binned_fill"]["streaming_bytes"]
        if st["record_passes"]:
            rec["binned_record"] = binned_record_bytes(st, c, bases, c["table_capacity"] * 8,
                                                       km["record"])
            rec["binned_record"]["direct_probe_bytes"] = alg["record"]
            alg["record"] = rec["binned_record"]["streaming_bytes"]
        rec["algorithmic_bytes"] = alg
        rec["roofline"] = roofline(alg, km, "primate_k25_%s" % ("blocked" if blocked else
                                                                "standard"))
    plan.close()
    torch.cuda.synchronize()
    return rec, d_in


def record_schedule_leg(args, stream):
    """The exact record, direct (random atomics into the table) and binned
    (tp_config.record_binned 2: candidates partitioned by home block, blocks
    built in LDS, as many passes as the scratch needs), on the primate
    workload at the given scales (8 genomes of 3 Gbp times the scale, filter
    bits scaled with them): record time, passes and whole-run time, mean of
    two runs after a warm-up run of each; the junction counts must agree."""
    import torch

    import paper_1602_05856_amd as tp
    import synth
    out = []
    for scale in [float(x) for x in args.record_scales.split(",") if x]:
        gs = synth.primate(0, scale, packed=True)
        genomes = [tp.Genome(packed=p, n_bases=m, n_runs=r) for p, m, r in gs]
        b = 1 << (PRIMATE_B_LOG2 + round(math.log2(scale)))
        plan = tp.Plan(genomes, PRIMATE_K, b, PRIMATE_H, tp.TP_FLAG_BLOCKED_FILTER)
        d_in = plan.upload()
        rec = {"scale": scale, "input_gbp": sum(m for _, m, _ in gs) / 1e9, "bloom_bits": b}
        for name, mode in (("direct", 1), ("binned", 2)):
            plan.config = {"record_binned": mode}
            plan.run(d_in, stream)  # warm-up: scratch and outputs sized
            per = []
            for _ in range(2):
                plan.run(d_in, stream)
                per.append(plan.stats())
            rec[name] = {"ms_record": sum(x["ms_record"] for x in per) / len(per),
                         "ms_total": sum(x["ms_total"] for x in per) / len(per),
                         "record_passes": per[-1]["record_passes"],
                         "junctions": per[-1]["junctions"],
                         "table_capacity": per[-1]["table_capacity"]}
        if rec["direct"]["junctions"] != rec["binned"]["junctions"]:
            raise SystemExit("record schedules disagree at scale %g" % scale)
        rec["record_speedup"] = rec["direct"]["ms_record"] / rec["binned"]["ms_record"]
        log("record schedules at scale %g: %s" % (scale, rec))
        plan.close()
        del d_in, gs, genomes
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out.append(rec)
    return out


def unpack_prefix(gs, per_genome):
    """Base codes (N = 4) of the first per_genome bases of each packed genome."""
    import numpy as np
    out = []
    for pk, m, runs in gs:
        n = min(int(m), per_genome)
        b = pk[:(n + 3) // 4]
        codes = np.stack([(b >> s) & 3 for s in (0, 2, 4, 6)], axis=1).reshape(-1)[:n]
        codes = codes.astype(np.uint8)
        for s, ln in runs:
            s, ln = int(s), int(ln)
            if s < n:
                codes[s:min(n, s + ln)] = 4
        out.append(codes)
    return out


def cpu_info():
    model = platform.processor() or ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)),
            "os_cpu_count": os.cpu_count()}


def cpu_baseline(gs, per_genome):
    """The C oracle (Algorithm 2, single-threaded) on a prefix of every genome
    of the headline workload, with its k, b, h and filter layout."""
    import oracle
    sample = unpack_prefix(gs, per_genome)
    bases = sum(int((c < 4).sum()) for c in sample)
    t0 = time.perf_counter()
    oracle.twopass(sample, PRIMATE_K, 1 << PRIMATE_B_LOG2, PRIMATE_H, blocked=True)
    dt = time.perf_counter() - t0
    del sample
    rec = {"value": bases / dt / 1e9, "unit": "Gbp/s", "cores": 1, "kind": "oracle",
           "sample": "first %d bases of each of the 8 primate-scale genomes (%.1f Mbp of "
                     "24 Gbp), same k=25, b=2^36, h=5 and blocked filter; single-threaded C "
                     "oracle, %.1f s" % (per_genome, bases / 1e6, dt)}
    rec.update(cpu_info())
    return rec


# --------------------------------------------------------------- bacterial

def bacterial_leg(args, stream):
    """The 62 x 5 Mbp workload (b = 2^30, h = 4): k = 25 blocked (tuned), the
    standard layout, and k = 63 / 100 blocked.  The 128 MiB filter sits in
    the last-level cache, so its probes cost no HBM bytes: its kernels are
    reported against the measured on-chip random-access rate instead."""
    import torch

    import paper_1602_05856_amd as tp
    import synth
    t0 = time.perf_counter()
    codes = synth.bacterial(0)
    bases = sum(int((c < 4).sum()) for c in codes)
    genomes = genomes_for(codes)
    log("bacterial workload: %d genomes, %.1f Mbp in %.1fs" % (
        len(codes), bases / 1e6, time.perf_counter() - t0))
    b, h = 1 << 30, 4
    out = {"workload": "62 bacterial genomes x 5 Mbp from one base, 0.5-2% SNPs, 0.2% indels, "
                       "repeat families; b=2^30, h=4", "input_mbp": bases / 1e6}
    d_in = None
    steps = max(3, args.steps // 2)
    for name, k, flags in (("k25_blocked", 25, tp.TP_FLAG_BLOCKED_FILTER), ("k25_standard", 25, 0),
                           ("k63_blocked", 63, tp.TP_FLAG_BLOCKED_FILTER),
                           ("k100_blocked", 100, tp.TP_FLAG_BLOCKED_FILTER)):
        if name not in args.bacterial_cases.split(","):
            continue
        plan = tp.Plan(genomes, k, b, h, flags)
        if d_in is None:
            d_in = plan.upload()
        tuned = tune(plan, d_in, args)
        ms, per = run_steps(plan, d_in, steps, 1, stream)
        st = per[-1]
        W = 1 if k <= 31 else (2 if k <= 63 else 4)
        km = kernel_avg(per)
        c = counts_of(st)
        nz = nonzero_granules_dev(plan.device_outputs()["bloom"], b // 32)
        alg, probes, where = algorithmic_bytes(c, bases, k, W, h, bool(flags), b // 8,
                                               c["table_capacity"] * slot_bytes(k, W), nz)
        rec = {"value": bases / 1e9 / (ms * 1e-3), "ms_per_step": ms, "kernel_ms": km,
               "tuned": tuned, "counts": c, "residency": where, "method_probes": probes,
               "roofline": roofline(alg, km, "bacterial_%s" % name)}
        if name == "k25_blocked" and args.h2h:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.upload_into(d_in, stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            plan.run(d_in, stream)
            t2 = time.perf_counter()
            res = plan.download(stream)
            t3 = time.perf_counter()
            rec["host_to_host"] = {
                "upload_ms": (t1 - t0) * 1e3, "run_ms": (t2 - t1) * 1e3,
                "download_ms": (t3 - t2) * 1e3, "gbps": bases / 1e9 / (t3 - t0),
                "result_mb": (res.junction_pos.nbytes + res.vertex.nbytes + res.strand.nbytes +
                              res.edges.nbytes) / 1e6}
            del res
        out[name] = rec
        log("bacterial %s: %.2f ms/step, %.2f Gbp/s, kernels %s" % (name, ms, rec["value"], km))
        plan.close()
    del d_in
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------- batched

def batched_leg(args, stream):
    """256 independent genome sets (log-uniform 50 kbp..20 Mbp, 2-10 genomes
    at 1% divergence), k = 31, h = 4, 16 filter bits per (k+1)-mer: one
    batched plan (one launch per phase over all sets, tuned), the same plan's
    whole run captured once as a HIP graph on caller memory and replayed,
    and one plan per set run back to back on the same stream."""
    import torch

    import paper_1602_05856_amd as tp
    import synth
    k, h = 31, 4
    flags = tp.TP_FLAG_BLOCKED_FILTER
    t0 = time.perf_counter()
    sets = synth.batched_sets(0, n_sets=args.sets)
    gsets = [genomes_for(c) for c in sets]
    bs = [tp.bloom_bits_for(g, k) for g in gsets]
    bases = sum(int((c < 4).sum()) for cs in sets for c in cs)
    log("batched workload: %d sets, %d genomes, %.1f Mbp in %.1fs" %
        (len(sets), sum(len(c) for c in sets), bases / 1e6, time.perf_counter() - t0))
    plan = tp.Plan.batch(list(zip(gsets, bs)), k, h, flags)
    d_in = plan.upload()
    tuned = tune(plan, d_in, args)
    steps = max(3, args.steps // 2)
    ms_b, per_b = run_steps(plan, d_in, steps, 1, stream)
    st = per_b[-1]
    km = kernel_avg(per_b)
    log("batched: %.2f ms/step, kernels %s" % (ms_b, km))

    # the whole batched run as one graph on caller memory (no host waits)
    L = plan.workspace_layout(args.graph_key_fraction, args.graph_key_fraction)
    ws, outb = plan.alloc_workspace()
    plan.prepare_workspace(ws, stream)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.run_ws(d_in, ws, outb, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.run_ws(d_in, ws, outb, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    cnt = plan.ws_counts(outb)
    assert cnt["status"] == 0 and cnt["junctions"] == st["junctions"], cnt
    t1 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    ms_g = (time.perf_counter() - t1) * 1e3 / steps
    log("batched, one graph: %.2f ms/step" % ms_g)
    del g, ws, outb
    plan.close()
    del d_in
    torch.cuda.empty_cache()

    plans = [tp.Plan(g_, k, b, h, flags) for g_, b in zip(gsets, bs)]
    ins = [p.upload() for p in plans]
    for p in plans:  # the batch's tuned grids and order; one-set table sizing
        p.config = {"wg_per_cu": tuned["wg_per_cu"], "tile_order": tuned["tile_order"]}
    for p, d in zip(plans, ins):
        p.run(d, stream)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        for p, d in zip(plans, ins):
            p.run(d, stream)
    torch.cuda.synchronize()
    ms_p = (time.perf_counter() - t2) * 1e3 / steps
    junctions_p = sum(p.stats()["junctions"] for p in plans)
    for p in plans:
        p.close()
    del ins
    torch.cuda.empty_cache()
    log("one set per launch: %.2f ms/step" % ms_p)
    assert junctions_p == st["junctions"], "batched and per-set junction counts differ"
    return {"workload": "%d sets, log-uniform 50 kbp..20 Mbp, 2-10 genomes at 1%% divergence, "
                        "k=%d, h=%d, 16 bits per (k+1)-mer, blocked filter" % (len(sets), k, h),
            "input_mbp": round(bases / 1e6, 3), "steps": steps,
            "batched_gbps": bases / 1e9 / (ms_b * 1e-3), "batched_ms": ms_b,
            "graph_gbps": bases / 1e9 / (ms_g * 1e-3), "graph_ms": ms_g,
            "graph_key_fraction": args.graph_key_fraction,
            "graph_workspace_gib": L["workspace_bytes"] / 2**30,
            "per_set_gbps": bases / 1e9 / (ms_p * 1e-3), "per_set_ms": ms_p,
            "speedup": ms_p / ms_b, "speedup_graph": ms_p / ms_g, "kernel_ms": km,
            "tuned": tuned, "chunk_tiles": tuned.get("chunk_tiles"),
            "counts": {n: st[n] for n in ("positions", "candidates", "junctions", "edges",
                                          "table_keys", "table_capacity", "table_attempts")}}


# ----------------------------------------------------------------- serving

def serving_leg(args):
    """Poisson arrivals of build requests drawn from the serving pool (8 sets
    of 1-5 Mbp at k = 25, 3 of 50-200 Mbp at k = 31, 3 of 1-3 Gbp at k = 63;
    70/25/5% of requests; h = 4, 16 filter bits per (k+1)-mer, blocked
    filter): the mix's capacity with every request submitted at once, then
    50% and 80% of it, and the same request list built one set per launch
    (one plan per request, back to back) for comparison."""
    import threading

    import numpy as np
    import torch

    import paper_1602_05856_amd as tp
    import synth
    r = np.random.default_rng(5)
    t0 = time.perf_counter()
    pool = {}
    for e in synth.serving_entries(0):
        name, k, i, glen, g = e
        gs = genomes_for(synth.serving_set(0, e))
        pool.setdefault(name, []).append((gs, tp.bloom_bits_for(gs, k), glen * g))
    log("serving pool generated in %.1fs" % (time.perf_counter() - t0))
    flags = tp.TP_FLAG_BLOCKED_FILTER
    classes = synth.SERVE_CLASSES
    shares = np.array([c[1] for c in classes])
    out = {"workload": "Poisson arrivals; 70% 1-5 Mbp (k=25), 25% 50-200 Mbp (k=31), "
                       "5% 1-3 Gbp (k=63) sets; h=4, 16 bits per (k+1)-mer, blocked filter; "
                       "inputs drawn from a pool of 8/3/3 sets per class",
           "requests": args.requests,
           "server": {"workers": args.serve_workers, "express_workers": args.serve_express,
                      "express_cus": args.serve_express_cus, "wg_per_cu": args.serve_wg,
                      "hbm_budget_gib": args.serve_budget_gib},
           "loads": []}

    def draw():
        reqs = []
        for _ in range(args.requests):
            ci = int(r.choice(len(classes), p=shares))
            name, _, _, k = classes[ci]
            gs, b, bases = pool[name][int(r.integers(len(pool[name])))]
            reqs.append((name, k, gs, b, bases))
        return reqs

    # one server for every pass, as a service runs: the saturated pass first
    # warms its workers' buffers, which then persist
    srv = tp.Server(hbm_budget=args.serve_budget_gib << 30, workers=args.serve_workers,
                    max_batch=32, batch_max_bases=20_000_000,
                    batch_total_bases=400_000_000, wg_per_cu=args.serve_wg,
                    express_workers=args.serve_express, express_cus=args.serve_express_cus)

    def run(reqs, gaps):
        batches0 = srv.stats()["batches"]
        ids = [None] * len(reqs)

        def submitter():
            start = time.perf_counter()
            due = 0.0
            for i, (name, k, gs, b, bases) in enumerate(reqs):
                if gaps is not None:
                    due += gaps[i]
                    delay = start + due - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                ids[i] = srv.submit(gs, k, b, 4, flags)

        th = threading.Thread(target=submitter)
        t_start = time.perf_counter()
        th.start()
        lat = []
        for i in range(len(reqs)):
            while ids[i] is None:
                time.sleep(0.0005)
            _, info = srv.wait(ids[i], keep=False)
            lat.append((reqs[i][0], info["end_s"] - info["submit_s"], info["batch_jobs"],
                        info["start_s"] - info["submit_s"], info["layout_ms"],
                        info["upload_ms"], info["run_ms"], info["download_ms"]))
        th.join()
        t_end = time.perf_counter()
        st = srv.stats()
        allv = np.array([x[1] for x in lat]) * 1e3
        rec = {"mean_job_mbp": sum(q[4] for q in reqs) / len(reqs) / 1e6,
               "p50_ms": float(np.percentile(allv, 50)), "p99_ms": float(np.percentile(allv, 99)),
               "aggregate_gbps": sum(q[4] for q in reqs) / 1e9 / (t_end - t_start),
               "batches": st["batches"] - batches0, "peak_held_gib": st["peak_held_bytes"] / 2**30,
               "per_class": {}}
        assert st["peak_held_bytes"] <= args.serve_budget_gib << 30
        for name, _, _, _ in classes:
            sel = [x for x in lat if x[0] == name]
            if not sel:
                continue
            v = np.array([x[1] for x in sel]) * 1e3
            rec["per_class"][name] = {
                "n": len(sel), "p50_ms": float(np.percentile(v, 50)),
                "p99_ms": float(np.percentile(v, 99)),
                "mean_queue_ms": float(np.mean([x[3] for x in sel]) * 1e3),
                "mean_upload_ms": float(np.mean([x[5] for x in sel])),
                "mean_run_ms": float(np.mean([x[6] for x in sel])),
                "mean_download_ms": float(np.mean([x[7] for x in sel]))}
        return rec

    reqs = draw()
    sat = run(reqs, None)
    cap = sat["aggregate_gbps"]
    out["capacity_gbps"] = cap
    out["saturated"] = sat
    log("serving, all submitted at once: %s" % sat)
    loads = []
    for frac in (0.5, 0.8):
        lreqs = draw()
        mean_bases = sum(q[4] for q in lreqs) / len(lreqs)
        qps = frac * cap * 1e9 / mean_bases
        rec = {"load": frac, "qps": qps}
        rec.update(run(lreqs, r.exponential(1.0 / qps, len(lreqs))))
        log("serving at %.0f%%: %s" % (100 * frac, rec))
        loads.append(rec)
    srv.close()
    out["loads"] = loads
    # the same request list, one plan per request built, uploaded, run and
    # downloaded in turn on one stream (its device buffers allocated per request)
    stream = torch.cuda.current_stream()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_class = {}
    for name, k, gs, b, bases in reqs:
        tq = [time.perf_counter()]
        p = tp.Plan(gs, k, b, 4, flags)
        d = p.upload(stream=stream)
        stream.synchronize()
        tq.append(time.perf_counter())
        p.run(d, stream)
        tq.append(time.perf_counter())
        res = p.download(stream)
        tq.append(time.perf_counter())
        del res, d
        p.close()
        tq.append(time.perf_counter())
        per_class.setdefault(name, []).append(np.diff(tq) * 1e3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    torch.cuda.empty_cache()
    out["one_set_per_launch_gbps"] = sum(q[4] for q in reqs) / 1e9 / dt
    out["one_set_per_launch_ms"] = {
        n: {"n": len(v), "mean": float(np.sum(v, axis=1).mean()),
            "max": float(np.sum(v, axis=1).max()),
            "mean_upload": float(np.mean([x[0] for x in v])),
            "mean_run": float(np.mean([x[1] for x in v])),
            "mean_download": float(np.mean([x[2] for x in v])),
            "mean_free": float(np.mean([x[3] for x in v]))}
        for n, v in per_class.items()}
    out["served_vs_one_set_per_launch"] = cap / out["one_set_per_launch_gbps"]
    log("serving: the same %d requests one plan per request: %.2f Gbp/s" % (
        len(reqs), out["one_set_per_launch_gbps"]))
    return out


# ------------------------------------------------------------ memory system

def membench_leg(args):
    """Random 8-byte accesses per second (loads, and the fill's one-bit
    atomic ORs) into device buffers of growing size: the rate the
    random-access kernels run against, from the on-chip caches (<= 256 MB)
    to HBM.  Plus a streaming device copy for the HBM bandwidth reference."""
    import torch

    import paper_1602_05856_amd as tp
    out = {"sizes": [], "unit": "G accesses/s"}
    ck = torch.zeros(1, dtype=torch.int64, device="cuda")
    for size in [int(x) << 20 for x in args.membench_mib.split(",")]:
        buf = torch.zeros(size, dtype=torch.uint8, device="cuda")
        rec = {"bytes": size}
        for mode, name in ((0, "load"), (1, "atomic_or")):
            tp.bench_random_access(buf, 1 << 26, mode, 7, ck)  # warm up (page mapping)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            n = tp.bench_random_access(buf, 1 << 31, mode, 11, ck)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            rec[name] = n / (ms * 1e-3) / 1e9
        out["sizes"].append(rec)
        log("random access into %.2f GiB: %.1f G loads/s, %.1f G atomics/s" % (
            size / 2**30, rec["load"], rec["atomic_or"]))
        del buf
        torch.cuda.empty_cache()
    src = torch.ones(4 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = 5 * 2 * src.numel() / (e0.elapsed_time(e1) * 1e-3) / 1e9
    log("device copy: %.0f GB/s (read + write)" % out["copy_gbs"])
    out["checksum"] = int(ck.item())
    del src, dst
    torch.cuda.empty_cache()
    return out


# ----------------------------------------------------------------- profiles

# kernels inside each timed phase of a run (the binned fill is five launches
# per chunk)
PROFILE_KERNELS = (("k_fill", "fill"), ("k_bin_count", "fill"), ("k_bin_scan", "fill"),
                   ("k_bin_scatter", "fill"), ("k_bin_split", "fill"), ("k_bin_apply", "fill"),
                   ("k_query", "query"), ("k_popcount", "query"),
                   ("k_record", "record"), ("k_rbin_", "record"),
                   ("k_decide", "decide"), ("k_emit", "compact"),
                   ("k_joff", "compact"), ("k_block_counts", "compact"),
                   ("k_scan_blocks", "compact"))


def profile_summary(tag, trace_dir, fetch_dir, write_dir, command):
    """Write profiles/kernels_<tag>.md and profiles/traffic_<tag>.txt from the
    CSV output of one rocprofv3 --kernel-trace --stats run and two --pmc runs
    (FETCH_SIZE, WRITE_SIZE) of the same command with --calibrate-copy.  The
    counters are scaled by what they read for the 256 MiB device copy and
    fill that --calibrate-copy adds.  Traffic is per run of each phase: the
    counters of all its kernels' dispatches over the number of runs (the
    query's dispatches; one per run of one round)."""
    import collections
    import csv

    def key_of(name):
        for pat, key in PROFILE_KERNELS:
            if "tp::" + pat in name:
                return key
        return None

    def counters(d):
        agg = collections.defaultdict(list)
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return agg

    def runs_of(agg):
        return max(1, sum(len(v) for n, v in agg.items() if "tp::k_query" in n))

    def first(d, pat):
        rows = [r for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv")))
                if pat in r["Kernel_Name"]]
        return float(min(rows, key=lambda r: int(r["Dispatch_Id"]))["Counter_Value"])

    stats = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_stats.csv"))))
    lines = ["# Kernel time: %s" % tag, "", "Command (from the repository root; rocprofv3 runs "
             "from /tmp with TMPDIR=/tmp):", "", "```", command, "```", "",
             "| kernel | calls | avg us | total % |", "|---|---|---|---|"]
    for r in stats[:16]:
        lines.append("| `%s` | %s | %.1f | %.2f |" % (r["Name"][:90], r["Calls"],
                                                      float(r["AverageNs"]) / 1e3,
                                                      float(r["Percentage"])))
    out = {"workload": tag, "source_digest": source_digest(), "kernels": {}}
    if fetch_dir != "-" and write_dir != "-":
        fe, wr = counters(fetch_dir), counters(write_dir)
        cal_fetch = first(fetch_dir, "copyBuffer")
        cal_write = first(write_dir, "FillFunctor")
        f_fac, w_fac = 262144.0 / cal_fetch, 262144.0 / cal_write
        per = collections.defaultdict(lambda: {"fetch_kib": 0.0, "write_kib": 0.0})
        for src, field in ((fe, "fetch_kib"), (wr, "write_kib")):
            runs = runs_of(src)
            for n, vs in src.items():
                k = key_of(n)
                if k:
                    per[k][field] += sum(vs) / runs
        out.update({"command_fetch": command.replace("--kernel-trace --stats",
                                                     "--pmc FETCH_SIZE").replace(trace_dir,
                                                                                 fetch_dir),
                    "command_write": command.replace("--kernel-trace --stats",
                                                     "--pmc WRITE_SIZE").replace(trace_dir,
                                                                                 write_dir),
                    "calibration": {"copy_256MiB_fetch_kib": cal_fetch,
                                    "fill_256MiB_write_kib": cal_write,
                                    "fetch_factor": f_fac, "write_factor": w_fac}})
        lines += ["", "## HBM traffic per run of each phase (rocprofv3 --pmc, scaled by a "
                  "256 MiB copy/fill)", "", "FETCH_SIZE factor %.3f (a 256 MiB device copy reads "
                  "back as %.0f KiB), WRITE_SIZE factor %.3f.  Random word accesses are 64-byte "
                  "requests, which FETCH_SIZE counts in full: for the random-access phases the "
                  "unscaled sum is the estimate." % (f_fac, cal_fetch, w_fac), "",
                  "| phase | FETCH KiB | WRITE KiB | unscaled GB/run | scaled GB/run |",
                  "|---|---|---|---|---|"]
        for k, v in per.items():
            b = v["fetch_kib"] * 1024 * f_fac + v["write_kib"] * 1024 * w_fac
            raw = (v["fetch_kib"] + v["write_kib"]) * 1024
            out["kernels"][k] = {"fetch_kib": v["fetch_kib"], "write_kib": v["write_kib"],
                                 "bytes_per_run": b, "raw_bytes_per_run": raw}
            lines.append("| %s | %.0f | %.0f | %.2f | %.2f |" % (
                k, v["fetch_kib"], v["write_kib"], raw / 1e9, b / 1e9))
        with open(os.path.join(PROFILES, "traffic_%s.txt" % tag), "w") as f:
            json.dump(out, f, indent=1)
    with open(os.path.join(PROFILES, "kernels_%s.md" % tag), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profile_requests(tag, pmc_dir, command):
    """Write profiles/requests_<tag>.md from one rocprofv3 --pmc run of
    TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_HIT_sum TCC_MISS_sum: the
    L2-to-fabric read requests of each kernel by size, and its L2 hit rate."""
    import collections
    import csv
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))):
        for pat, _ in PROFILE_KERNELS:
            if "tp::" + pat + "<" in r["Kernel_Name"] or "tp::" + pat + "(" in r["Kernel_Name"]:
                agg[pat][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["# L2-to-fabric read requests by size: %s" % tag, "",
             "Command (from the repository root; rocprofv3 runs from /tmp with TMPDIR=/tmp):",
             "", "```", command, "```", "", "Per launch (average over the launches of the run):",
             "", "| kernel | EA read requests | of which 32 B | L2 hits | L2 misses | L2 hit rate "
             "| requests x 64 B (GB) |", "|---|---|---|---|---|---|---|"]
    any32 = 0.0
    for pat, _ in PROFILE_KERNELS:
        if pat not in agg:
            continue
        c = {n: sum(v) / len(v) for n, v in agg[pat].items()}
        req, r32 = c.get("TCC_EA0_RDREQ_sum", 0.0), c.get("TCC_EA0_RDREQ_32B_sum", 0.0)
        hit, miss = c.get("TCC_HIT_sum", 0.0), c.get("TCC_MISS_sum", 0.0)
        any32 += r32
        lines.append("| %s | %.3g | %.3g | %.3g | %.3g | %.0f%% | %.2f |" % (
            pat, req, r32, hit, miss, 100 * hit / max(1.0, hit + miss), req * 64 / 1e9))
    lines += ["", ("No kernel issues a 32-byte read request, so a random word access moves at "
                   "least 64 bytes: the granule of the algorithmic byte model." if any32 == 0 else
                   "Some kernels issue 32-byte read requests (column 3).")]
    with open(os.path.join(PROFILES, "requests_%s.md" % tag), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


# -------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps of the headline")
    ap.add_argument("--warmup", type=int, default=2, help="untimed headline steps first")
    ap.add_argument("--primate", type=int, default=1,
                    help="0 = skip the headline and print only the other legs' record "
                         "(for profiling one leg)")
    ap.add_argument("--primate-load", type=float, default=0.7,
                    help="exact-table load target of the primate workload")
    ap.add_argument("--primate-rounds", type=int, default=1)
    ap.add_argument("--primate-standard", type=int, default=1,
                    help="timed steps of the standard filter layout on the primate input (0 = skip)")
    ap.add_argument("--bacterial", type=int, default=1, help="the 62 x 5 Mbp leg (0 = skip)")
    ap.add_argument("--bacterial-cases", default="k25_blocked,k25_standard,k63_blocked,k100_blocked")
    ap.add_argument("--sets", type=int, default=256, help="sets of the batched leg (0 = skip)")
    ap.add_argument("--graph-key-fraction", type=float, default=0.25,
                    help="table bound (distinct candidate k-mers per position) of the graph run")
    ap.add_argument("--requests", type=int, default=300,
                    help="requests per load level of the serving leg (0 = skip)")
    ap.add_argument("--serve-workers", type=int, default=3)
    ap.add_argument("--serve-express", type=int, default=1)
    ap.add_argument("--serve-budget-gib", type=int, default=200)
    ap.add_argument("--serve-wg", type=int, default=4)
    ap.add_argument("--serve-express-cus", type=int, default=32,
                    help="CUs kept for the express worker's kernels (0 = shared)")
    ap.add_argument("--membench", type=int, default=1, help="random-access rates (0 = skip)")
    ap.add_argument("--record-scales", default="",
                    help="primate scales at which to time the direct against the binned "
                         "record, e.g. 0.25,0.5,1 (empty = skip)")
    ap.add_argument("--membench-mib", default="64,128,256,512,1024,8192,65536")
    ap.add_argument("--cpu-prefix", type=int, default=500_000,
                    help="bases per genome of the oracle's CPU sample (0 = skip)")
    ap.add_argument("--tune", type=int, default=1)
    ap.add_argument("--config", default=None)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--h2h", type=int, default=1,
                    help="time one host-to-host run of the bacterial workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB fill and copy (scales the FETCH_SIZE / "
                         "WRITE_SIZE counters of a profiled run)")
    ap.add_argument("--profile-summary", nargs=5,
                    metavar=("TAG", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="summarize rocprofv3 CSV output into profiles/ and exit (no GPU); "
                         "FETCH_DIR and WRITE_DIR may be '-'")
    ap.add_argument("--profile-requests", nargs=3, metavar=("TAG", "PMC_DIR", "COMMAND"),
                    help="summarize a rocprofv3 --pmc run of the L2 read-request counters "
                         "into profiles/requests_TAG.md and exit (no GPU)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(*args.profile_summary)
        return
    if args.profile_requests:
        profile_requests(*args.profile_requests)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1602_05856_amd as tp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tp.lib()  # fails loudly when the HIP library is missing
    stream = torch.cuda.current_stream()
    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if not args.primate:
        # the other legs alone (a profile of one of them): no headline line
        out = {"bacterial": bacterial_leg(args, stream) if args.bacterial else None,
               "batched": batched_leg(args, stream) if args.sets > 0 else None,
               "serving": serving_leg(args) if args.requests > 0 else None,
               "membench": membench_leg(args) if args.membench else None,
               "record_schedules": record_schedule_leg(args, stream) if args.record_scales
               else None,
               "source_digest": source_digest()}
        print(json.dumps(out), flush=True)
        return
    gs, genomes, bases = primate_input()
    head, d_in = primate_leg(args, stream, genomes, bases, tp.TP_FLAG_BLOCKED_FILTER,
                             args.steps, args.warmup)
    log("primate blocked: %.1f ms/step, %.2f Gbp/s, kernels %s, roofline %s" % (
        head["ms_per_step"], head["value"], head["kernel_ms"], head["roofline"]))
    standard = None
    if args.primate_standard:
        standard, _ = primate_leg(args, stream, genomes, bases, 0, args.primate_standard, 0,
                                  d_in=d_in, order=head["config"]["pass2_slabs"])
        log("primate standard: %.1f ms/step, %.2f Gbp/s" % (standard["ms_per_step"],
                                                            standard["value"]))
    del d_in
    torch.cuda.empty_cache()
    cpu = cpu_baseline(gs, args.cpu_prefix) if args.cpu_prefix else None
    if cpu:
        log("cpu baseline %s" % cpu)
    del gs, genomes
    bacterial = bacterial_leg(args, stream) if args.bacterial else None
    batched = batched_leg(args, stream) if args.sets > 0 else None
    serving = serving_leg(args) if args.requests > 0 else None
    mem = membench_leg(args) if args.membench else None
    schedules = record_schedule_leg(args, stream) if args.record_scales else None
    if mem:
        # the headline kernels' random-access rates against the measured ceiling
        sizes = mem["sizes"]

        def ceiling(nbytes, kind):
            fit = [s for s in sizes if s["bytes"] >= nbytes] or sizes[-1:]
            return fit[0][kind]

        c = head["counts"]
        filt, table = (1 << PRIMATE_B_LOG2) // 8, c["table_capacity"] * 8
        # (a binned fill or record makes no random accesses: each has its own
        # streaming entry, binned_fill and binned_record)
        head["random_access"] = {
            n: {"g_per_s": head["method_probes"][n] / (head["kernel_ms"][n] * 1e-3) / 1e9,
                "ceiling_g_per_s": ceiling(filt if n in ("fill", "query") else table,
                                           "atomic_or" if n in ("fill", "record") else "load")}
            for n in ("fill", "query", "record", "decide")
            if not (n == "fill" and "binned_fill" in head)
            and not (n == "record" and "binned_record" in head)}
        for v in head["random_access"].values():
            v["frac_of_ceiling"] = v["g_per_s"] / v["ceiling_g_per_s"]

    line = {
        "metric": "input Gbp/s for junction finding (pass1+pass2)",
        "value": head["value"],
        "unit": "Gbp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "8 primate-scale genomes x 3 Gbp from one base, 1-8% pairwise "
                               "divergence, indels, 300 bp and 6 kbp repeat families, N runs; "
                               "k=25, b=2^36, h=5, blocked filter, one round",
                   "input_gbp": round(bases / 1e9, 4), "k": PRIMATE_K,
                   "bloom_bits": 1 << PRIMATE_B_LOG2, "hashes": PRIMATE_H, "filter": "blocked"},
        "pass12_gbps": bases / 1e9 / (head["pass12_ms"] * 1e-3),
        "kernel_ms": head["kernel_ms"],
        "counts": head["counts"],
        "roofline": head["roofline"],
        "primate": head,
        "primate_standard": standard,
        "bacterial": bacterial,
        "batched": batched,
        "serving": serving,
        "membench": mem,
        "record_schedules": schedules,
        "cpu_baseline": cpu,
        "source_digest": source_digest(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
