#!/usr/bin/env python3
"""Junction-finding throughput on one MI355X.

Workload: 62 bacterial-sized genomes (5 Mbp each, ~310 Mbp) derived from one
random base genome with 0.5-2% SNPs, 0.2% indels and 50 two-copy repeat
families; k = 25, Bloom filter 2^30 bits, 4 hash functions.  Synthetic
stand-in for the 62 E. coli benchmark of the paper's Results section.

A step is one pass of the whole device path over the resident packed input:
sentinels, Bloom fill, Bloom query (candidates), exact-table record,
junction decision, ordered compaction and compacted edges.  The metric is
input gigabases per second (non-N bases / step time).  The headline uses the
blocked filter layout; the standard layout is timed beside it.  Prints one
JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
GRANULE = 64            # bytes the memory system moves per random word access: every
                        # L2-to-fabric read request of these kernels is 64 B or more
                        # (rocprofv3 TCC_EA0_RDREQ_32B_sum = 0), so no access costs less
PROFILES = os.path.join(ROOT, "profiles")


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


def algorithmic_bytes(st, bases, k, W, nonzero_granules):
    """Bytes each kernel must move (the direct-probe model): the genome
    streamed at 2 bits per base, position bitmaps at 1 bit per position,
    outputs as written, and one GRANULE per random filter or table access
    the method makes: per filter probe read, per filter granule left
    non-zero (written once), and per table array an insert or lookup touches
    (1 packed, 2 split key/mask, 2-3 two-word keys, 3-4 four-word keys: top
    word, lower words, and a mask array unless the mask fits in the top
    word)."""
    pos, cand, nj, ne = st["positions"], st["candidates"], st["junctions"], st["edges"]
    genome = bases / 4
    if k <= 27:
        arrays = 1
    elif W == 1:
        arrays = 2
    else:
        himask = 2 * k <= 64 * (W - 1) + 54
        arrays = (2 if W == 2 else 3) + (0 if himask else 1)
    return {
        "fill": genome + GRANULE * (st["fill_loads"] + nonzero_granules),
        "query": genome + pos / 8 + GRANULE * st["query_probes"],
        "record": genome + pos / 8 + GRANULE * arrays * cand,
        "decide": genome + 2 * pos / 8 + GRANULE * arrays * cand,
        # bitmap read once, the k-mers at junctions from the packed genome,
        # junctions and edges written
        "compact": pos / 8 + genome + nj * (8 + 8 * W + 1) + ne * 24,
    }


def nonzero_granules(plan):
    """Filter granules (GRANULE bytes) with any bit set after the fill."""
    import numpy as np
    words = plan.debug_bloom()
    g = words.reshape(-1, GRANULE // 4) if words.size * 4 >= GRANULE else words.reshape(1, -1)
    return int(np.count_nonzero(g.any(axis=1)))


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1602_05856_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, filt, k):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(PROFILES, "traffic_bacterial_k%d_%s.txt" % (k, filt))
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest():
        return None, None
    kr = rec.get("kernels", {}).get(kernel, {})
    return kr.get("bytes_per_launch"), kr.get("raw_bytes_per_launch")


def tune(plan, d_in, args):
    """Autotune the plan's runtime knobs (outside the timed region), or apply
    the ones given with --config."""
    if args.config:
        plan.config = json.loads(args.config)
        return plan.config
    if not args.tune:
        return plan.config
    t0 = time.perf_counter()
    cfg = plan.autotune(d_in, args.tune_cache)
    log("autotuned in %.1fs: %s" % (time.perf_counter() - t0, cfg))
    return cfg


def run_steps(plan, d_in, steps, warmup, stream):
    import torch
    for i in range(warmup):
        plan.run(d_in, stream)
        log("warmup %d: %.2f ms" % (i, plan.stats()["ms_total"]))
    torch.cuda.synchronize()
    per_step = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(d_in, stream)
        per_step.append(plan.stats())
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, per_step


def batched_leg(args, stream):
    """Batched workload: independent genome sets of uneven size (total
    log-uniform in 50 kbp..20 Mbp, 2-10 related genomes each), k=31, h=4,
    16 filter bits per (k+1)-mer per set.  Times the sets as one batched plan
    (each phase one launch over all sets) and as one plan per set run back to
    back on the same stream (three host waits per set), inputs resident."""
    import paper_1602_05856_amd as tp
    import synth
    k, h = 31, 4
    flags = tp.TP_FLAG_BLOCKED_FILTER if args.filter == "blocked" else 0
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
    kernel_ms = {n: sum(x["ms_" + n] for x in per_b) / len(per_b)
                 for n in ("fill", "query", "record", "decide", "compact")}
    log("batched: %.2f ms/step, kernels %s" % (ms_b, kernel_ms))
    plan.close()
    del d_in

    import torch
    plans = [tp.Plan(g, k, b, h, flags) for g, b in zip(gsets, bs)]
    ins = [p.upload() for p in plans]

    def per_set(graphs):
        for p in plans:  # the batch's tuned grids and order; one-set table sizing
            p.config = {"wg_per_cu": tuned["wg_per_cu"], "tile_order": tuned["tile_order"],
                        "graphs": graphs}
        for p, d in zip(plans, ins):
            p.run(d, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            for p, d in zip(plans, ins):
                p.run(d, stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3 / steps

    ms_p = per_set(0)
    ms_pg = per_set(1)
    log("one set per launch, graphs: %.2f ms/step" % ms_pg)
    ms_p = min(ms_p, ms_pg)  # the faster form is the baseline
    junctions_p = sum(p.stats()["junctions"] for p in plans)
    for p in plans:
        p.close()
    log("one set per launch: %.2f ms/step" % ms_p)
    assert junctions_p == st["junctions"], "batched and per-set junction counts differ"
    return {"workload": "%d sets, log-uniform 50 kbp..20 Mbp, 2-10 genomes at 1%% divergence, "
                        "k=%d, h=%d, 16 bits per (k+1)-mer, %s filter" % (len(sets), k, h, args.filter),
            "input_mbp": round(bases / 1e6, 3), "steps": steps,
            "batched_gbps": bases / 1e9 / (ms_b * 1e-3), "batched_ms": ms_b,
            "per_set_gbps": bases / 1e9 / (ms_p * 1e-3), "per_set_ms": ms_p,
            "per_set_graphs_ms": ms_pg,
            "speedup": ms_p / ms_b, "kernel_ms": kernel_ms, "tuned": tuned,
            "counts": {n: st[n] for n in ("positions", "candidates", "junctions", "edges",
                                          "table_keys", "table_capacity", "table_attempts")}}


SERVE_CLASSES = (  # name, share, set size range (bases), k
    ("small", 0.70, (1e6, 5e6), 25),
    ("medium", 0.25, (50e6, 200e6), 31),
    ("large", 0.05, (1e9, 3e9), 63),
)


def serving_leg(args, capacity_gbps):
    """Serving workload: Poisson arrivals of build requests, 70% 1-5 Mbp sets
    at k=25, 25% 50-200 Mbp at k=31 and 5% 1-3 Gbp at k=63 (2-10 related
    genomes each, h=4, 16 filter bits per (k+1)-mer), at 50% and 80% of the
    mix's capacity, measured first by submitting every request at once (the
    large k=63 jobs carry most of the bases, so the mix's capacity is well
    below the batched k=31 one).  Requests draw their inputs from a pool
    generated once per class (jobs are independent, so reuse changes no
    work).  Reports p50/p99 job latency (submit to result on the host) and
    aggregate Gbp/s."""
    import threading

    import numpy as np

    import paper_1602_05856_amd as tp
    import synth
    r = np.random.default_rng(5)
    t0 = time.perf_counter()
    pool = {}
    for ci, (name, share, (lo, hi), k) in enumerate(SERVE_CLASSES):
        n = {"small": 8, "medium": 3, "large": 1}[name]
        entries = []
        for i in range(n):
            total = float(np.exp(r.uniform(np.log(lo), np.log(hi))))
            g = int(r.integers(2, 11))
            codes = synth.genome_set(synth.rng(5, ci, i), int(total / g), g)
            gs = genomes_for(codes)
            entries.append((gs, tp.bloom_bits_for(gs, k), sum(int(c.size) for c in codes)))
            del codes
        pool[name] = entries
    log("serving pool generated in %.1fs" % (time.perf_counter() - t0))
    flags = tp.TP_FLAG_BLOCKED_FILTER if args.filter == "blocked" else 0
    shares = np.array([c[1] for c in SERVE_CLASSES])
    out = {"workload": "Poisson arrivals; 70%% 1-5 Mbp (k=25), 25%% 50-200 Mbp (k=31), "
                       "5%% 1-3 Gbp (k=63) sets; h=4, 16 bits per (k+1)-mer, %s filter; "
                       "inputs drawn from a pool of 8/3/1 sets per class" % args.filter,
           "requests": args.requests, "batched_capacity_gbps": capacity_gbps,
           "server": {"workers": args.serve_workers, "express_workers": args.serve_express,
                      "wg_per_cu": args.serve_wg}, "loads": []}

    def draw():
        reqs = []
        for _ in range(args.requests):
            ci = int(r.choice(len(SERVE_CLASSES), p=shares))
            name, _, _, k = SERVE_CLASSES[ci]
            gs, b, bases = pool[name][int(r.integers(len(pool[name])))]
            reqs.append((name, k, gs, b, bases))
        return reqs

    def run(reqs, gaps):
        """Submit reqs (gaps between arrivals; None: all at once) and time them."""
        srv = tp.Server(hbm_budget=args.serve_budget_gib << 30, workers=args.serve_workers,
                        max_batch=32, batch_max_bases=20_000_000,
                        batch_total_bases=400_000_000, wg_per_cu=args.serve_wg,
                        express_workers=args.serve_express)
        ids = [None] * len(reqs)
        wall = {}

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
            wall["submitted"] = time.perf_counter()

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
        srv.close()
        allv = np.array([x[1] for x in lat]) * 1e3
        rec = {"mean_job_mbp": sum(q[4] for q in reqs) / len(reqs) / 1e6,
               "p50_ms": float(np.percentile(allv, 50)), "p99_ms": float(np.percentile(allv, 99)),
               "aggregate_gbps": sum(q[4] for q in reqs) / 1e9 / (t_end - t_start),
               "batches": st["batches"], "peak_held_gib": st["peak_held_bytes"] / 2**30,
               "per_class": {}}
        for name, _, _, _ in SERVE_CLASSES:
            sel = [x for x in lat if x[0] == name]
            if not sel:
                continue
            v = np.array([x[1] for x in sel]) * 1e3
            rec["per_class"][name] = {
                "n": len(sel), "p50_ms": float(np.percentile(v, 50)),
                "p99_ms": float(np.percentile(v, 99)),
                "mean_queue_ms": float(np.mean([x[3] for x in sel]) * 1e3),
                "mean_layout_ms": float(np.mean([x[4] for x in sel])),
                "mean_upload_ms": float(np.mean([x[5] for x in sel])),
                "mean_run_ms": float(np.mean([x[6] for x in sel])),
                "mean_download_ms": float(np.mean([x[7] for x in sel]))}
        return rec

    # the mix's own capacity: every request submitted at once
    sat = run(draw(), None)
    cap = sat["aggregate_gbps"]
    out["capacity_gbps"] = cap
    out["saturated"] = sat
    log("serving, all submitted at once: %s" % sat)
    for frac in (0.5, 0.8):
        reqs = draw()
        mean_bases = sum(q[4] for q in reqs) / len(reqs)
        qps = frac * cap * 1e9 / mean_bases
        rec = {"load": frac, "qps": qps}
        rec.update(run(reqs, r.exponential(1.0 / qps, len(reqs))))
        log("serving at %.0f%%: %s" % (100 * frac, rec))
        out["loads"].append(rec)
    return out


def cpu_baseline(codes, k, b, h, n_sample, blocked):
    import oracle
    sample = codes[:n_sample]
    bases = sum(int((c < 4).sum()) for c in sample)
    t0 = time.perf_counter()
    oracle.twopass(sample, k, b, h, blocked=blocked)
    dt = time.perf_counter() - t0
    return {"value": bases / dt / 1e9, "unit": "Gbp/s", "cores": 1, "kind": "oracle",
            "sample": "first %d of the %d genomes (%.1f Mbp), same k, b, h and filter; "
                      "single-threaded C oracle, %.1f s" % (n_sample, len(codes), bases / 1e6, dt)}


def primate_leg(args, stream, base_cfg=None):
    """Primate-scale workload (8 genomes of 3 Gbp; k=25, b=2^36, h=5): the
    memory-bound case, whose 8 GiB filter does not fit the on-chip caches.
    Timed with the blocked filter (the benchmarked layout) and the standard
    one, at the headline's tuned workgroup counts and the faster of two pass-2
    tile orders (the full tuner would take ~30 full runs), in one round at
    the default table load target (0.7: ~1.14e10 slots, 91 GB, beside ~171 GB
    of outputs)."""
    import torch

    import paper_1602_05856_amd as tp
    import synth
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    gs = synth.primate(0, 1.0, packed=True)
    bases = sum(int(m) - int(r[:, 1].sum()) for _, m, r in gs)
    genomes = [tp.Genome(packed=p, n_bases=m, n_runs=r) for p, m, r in gs]
    log("primate workload: %d genomes, %.2f Gbp (%.2f Gbp without N) in %.1fs" % (
        len(gs), sum(m for _, m, _ in gs) / 1e9, bases / 1e9, time.perf_counter() - t0))
    out = {"workload": "8 primate-scale genomes of 3 Gbp from one base, 1-8% pairwise "
                       "divergence, indels, 300 bp and 6 kbp repeat families, N runs; k=25, "
                       "b=2^36, h=5", "input_gbp": bases / 1e9, "rounds": args.primate_rounds,
           "table_load": args.primate_load}
    d_in = None
    order = None
    for name, flags in (("blocked", tp.TP_FLAG_BLOCKED_FILTER), ("standard", 0)):
        plan = tp.Plan(genomes, 25, 1 << 36, 5, flags)
        if d_in is None:
            d_in = plan.upload()
        plan.rounds = args.primate_rounds
        plan.config = {"table_load": args.primate_load}
        if base_cfg:
            plan.config = {"wg_per_cu": base_cfg["wg_per_cu"]}
        if order is None:
            # the pass-2 tile order, from one run of each (homologous tiles of
            # 3 Gbp genomes drift apart by indels, unlike the 5 Mbp ones)
            t = {}
            for ps in (2, 0):
                plan.config = {"pass2_slabs": ps}
                plan.run(d_in, stream)
                st = plan.stats()
                t[ps] = st["ms_record"] + st["ms_decide"]
            order = min(t, key=t.get)
        plan.config = {"pass2_slabs": order}
        ms, per = run_steps(plan, d_in, args.primate_steps, 0, stream)
        st = per[-1]
        out[name] = {"value": bases / 1e9 / (ms * 1e-3), "ms_per_step": ms,
                     "config": plan.config,
                     "kernel_ms": {kk: sum(s["ms_" + kk] for s in per) / len(per)
                                   for kk in ("fill", "query", "record", "decide", "compact")},
                     "counts": {kk: st[kk] for kk in ("candidates", "junctions", "edges",
                                                      "table_keys", "table_capacity")}}
        log("primate %s: %s" % (name, out[name]))
        plan.close()
    del d_in
    torch.cuda.empty_cache()
    return out


PROFILE_KERNELS = (("k_fill", "fill"), ("k_query", "query"), ("k_popcount", "query"),
                   ("k_record", "record"), ("k_decide", "decide"), ("k_emit", "compact"),
                   ("k_joff", "compact"), ("k_block_counts", "compact"),
                   ("k_scan_blocks", "compact"))


def profile_summary(tag, trace_dir, fetch_dir, write_dir, command):
    """Write profiles/kernels_<tag>.md and profiles/traffic_<tag>.txt from the
    CSV output of one rocprofv3 --kernel-trace --stats run and two --pmc runs
    (FETCH_SIZE, WRITE_SIZE) of the same command with --calibrate-copy.  The
    counters are scaled by what they read for the 256 MiB device copy and
    fill that --calibrate-copy adds."""
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

    def first(d, pat):
        # the calibration copy and fill are the run's first dispatches of their kind
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
    fe, wr = counters(fetch_dir), counters(write_dir)
    cal_fetch = first(fetch_dir, "copyBuffer")
    cal_write = first(write_dir, "FillFunctor")
    f_fac, w_fac = 262144.0 / cal_fetch, 262144.0 / cal_write
    per = collections.defaultdict(lambda: {"fetch_kib": 0.0, "write_kib": 0.0})
    for src, field in ((fe, "fetch_kib"), (wr, "write_kib")):
        for n, vs in src.items():
            k = key_of(n)
            if k:
                per[k][field] += sum(vs) / len(vs)
    out = {"workload": tag,
           "command_fetch": command.replace("--kernel-trace --stats", "--pmc FETCH_SIZE")
                                   .replace(trace_dir, fetch_dir),
           "command_write": command.replace("--kernel-trace --stats", "--pmc WRITE_SIZE")
                                   .replace(trace_dir, write_dir),
           "source_digest": source_digest(),
           "calibration": {"copy_256MiB_fetch_kib": cal_fetch, "fill_256MiB_write_kib": cal_write,
                           "fetch_factor": f_fac, "write_factor": w_fac},
           "kernels": {}}
    lines += ["", "## HBM traffic per launch (rocprofv3 --pmc, scaled by a 256 MiB copy/fill)",
              "", "FETCH_SIZE factor %.3f (a 256 MiB device copy reads back as %.0f KiB), "
              "WRITE_SIZE factor %.3f." % (f_fac, cal_fetch, w_fac), "",
              "| kernel | FETCH KiB | WRITE KiB | scaled GB/launch |", "|---|---|---|---|"]
    for k, v in per.items():
        b = v["fetch_kib"] * 1024 * f_fac + v["write_kib"] * 1024 * w_fac
        out["kernels"][k] = {"fetch_kib": v["fetch_kib"], "write_kib": v["write_kib"],
                             "bytes_per_launch": b,
                             "raw_bytes_per_launch": (v["fetch_kib"] + v["write_kib"]) * 1024}
        lines.append("| %s | %.0f | %.0f | %.2f |" % (k, v["fetch_kib"], v["write_kib"], b / 1e9))
    with open(os.path.join(PROFILES, "kernels_%s.md" % tag), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(PROFILES, "traffic_%s.txt" % tag), "w") as f:
        json.dump(out, f, indent=1)
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=int, default=25)
    ap.add_argument("--bloom-log2", type=int, default=30)
    ap.add_argument("--hashes", type=int, default=4)
    ap.add_argument("--genomes", type=int, default=62)
    ap.add_argument("--filter", choices=("standard", "blocked"), default="blocked",
                    help="first-pass Bloom filter layout of the headline")
    ap.add_argument("--compare", type=int, default=1,
                    help="also time the other filter layout (0 = skip)")
    ap.add_argument("--cpu-sample", type=int, default=2,
                    help="genomes in the CPU-oracle baseline sample (0 = skip)")
    ap.add_argument("--tune", type=int, default=1,
                    help="autotune each plan's runtime knobs before timing (0 = defaults)")
    ap.add_argument("--config", default=None,
                    help='headline plan knobs as JSON, e.g. \'{"wg_per_cu": [0, 0, 6, 6]}\' '
                         "(skips the autotuner; for profiling a fixed configuration)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (default: none, tune every run)")
    ap.add_argument("--long-k", type=int, default=100,
                    help="also time the headline input at this k > 63 (0 = skip)")
    ap.add_argument("--rounds", type=int, default=4,
                    help="also time Algorithm 3 with this many rounds (1 = skip)")
    ap.add_argument("--sets", type=int, default=256,
                    help="genome sets of the batched leg (0 = skip it)")
    ap.add_argument("--requests", type=int, default=200,
                    help="requests per load level of the serving leg (0 = skip it)")
    ap.add_argument("--serve-workers", type=int, default=3)
    ap.add_argument("--serve-express", type=int, default=1,
                    help="of the serving workers, how many take only small jobs")
    ap.add_argument("--serve-budget-gib", type=int, default=200)
    ap.add_argument("--serve-wg", type=int, default=4,
                    help="workgroups per CU of each served job's kernels (0 = all that fit)")
    ap.add_argument("--primate", type=int, default=1,
                    help="also time the 8 x 3 Gbp primate-scale workload (k=25, b=2^36, h=5)")
    ap.add_argument("--primate-rounds", type=int, default=1)
    ap.add_argument("--primate-load", type=float, default=0.7,
                    help="exact-table load target of the primate leg")
    ap.add_argument("--primate-steps", type=int, default=2)
    ap.add_argument("--h2h", type=int, default=1,
                    help="also time one host-to-host run (upload, run, download)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 256 MiB fill and copy (known-size kernels that scale "
                         "the FETCH_SIZE / WRITE_SIZE counters of a profiled run)")
    ap.add_argument("--profile-summary", nargs=5,
                    metavar=("TAG", "TRACE_DIR", "FETCH_DIR", "WRITE_DIR", "COMMAND"),
                    help="summarize rocprofv3 CSV output into profiles/ and exit (no GPU)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(*args.profile_summary)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1602_05856_amd as tp
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tp.lib()  # fails loudly when the HIP library is missing
    k, b, h = args.k, 1 << args.bloom_log2, args.hashes
    W = 1 if k <= 31 else (2 if k <= 63 else 4)
    t0 = time.perf_counter()
    codes = synth.bacterial(0, n_genomes=args.genomes)
    bases = sum(int((c < 4).sum()) for c in codes)
    genomes = genomes_for(codes)
    log("generated %d genomes, %.1f Mbp in %.1fs" % (len(codes), bases / 1e6,
                                                      time.perf_counter() - t0))
    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()

    def plan_for(filt):
        flags = tp.TP_FLAG_BLOCKED_FILTER if filt == "blocked" else 0
        return tp.Plan(genomes, k, b, h, flags)

    plan = plan_for(args.filter)
    d_in = plan.upload()
    tuned = tune(plan, d_in, args)
    ms_per_step, per_step = run_steps(plan, d_in, args.steps, args.warmup, stream)

    def avg(key):
        return sum(s[key] for s in per_step) / len(per_step)

    kernel_ms = {"fill": avg("ms_fill"), "query": avg("ms_query"), "record": avg("ms_record"),
                 "decide": avg("ms_decide"), "compact": avg("ms_compact")}
    st = dict(per_step[-1])
    st["fill_loads"] = st["edge_positions"] * (1 if args.filter == "blocked" else h)
    alg = algorithmic_bytes(st, bases, k, W, nonzero_granules(plan))
    dom = max(kernel_ms, key=lambda n: kernel_ms[n])
    achieved = alg[dom] / (kernel_ms[dom] * 1e-3) / 1e9
    log("step %.2f ms; kernels %s; stats %s" % (ms_per_step, kernel_ms, st))
    # host to host: packed genomes copied in, the path run, the result copied out
    host = None
    if args.h2h:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.upload_into(d_in, stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.run(d_in, stream)
        t2 = time.perf_counter()
        res = plan.download(stream)
        t3 = time.perf_counter()
        host = {"upload_ms": (t1 - t0) * 1e3, "run_ms": (t2 - t1) * 1e3,
                "download_ms": (t3 - t2) * 1e3,
                "result_mb": (res.junction_pos.nbytes + res.vertex.nbytes + res.strand.nbytes +
                              res.edges.nbytes) / 1e6}
        host["gbps"] = bases / 1e9 / ((t3 - t0))
        log("host to host: %s" % host)
        del res
    plan.close()

    rounds_leg = None
    if args.rounds > 1:
        # Algorithm 3 on the same input: the peak exact table shrinks with the
        # number of rounds, at the cost of a pass over the input per round
        p3 = plan_for(args.filter)
        p3.config = tuned
        p3.rounds = args.rounds
        ms3, per3 = run_steps(p3, d_in, max(3, args.steps // 2), 1, stream)
        rounds_leg = {"rounds": args.rounds, "value": bases / 1e9 / (ms3 * 1e-3),
                      "ms_per_step": ms3, "candidates": per3[-1]["candidates"],
                      "junctions": per3[-1]["junctions"],
                      "table_capacity_per_round": per3[-1]["table_capacity"],
                      "table_capacity_one_round": st["table_capacity"],
                      "kernel_ms": {n: sum(x["ms_" + n] for x in per3) / len(per3)
                                    for n in ("fill", "query", "record", "decide", "compact")}}
        assert rounds_leg["junctions"] == st["junctions"], "rounds changed the junctions"
        log("rounds %s" % rounds_leg)
        p3.close()

    long_k = None
    if args.long_k:
        # the paper's second k (Results section): four-word k-mers, same input
        p4 = tp.Plan(genomes, args.long_k, b, h,
                     tp.TP_FLAG_BLOCKED_FILTER if args.filter == "blocked" else 0)
        cfg4 = tune(p4, d_in, args) if not args.config else p4.config
        ms4, per4 = run_steps(p4, d_in, max(3, args.steps // 2), 1, stream)
        long_k = {"k": args.long_k, "value": bases / 1e9 / (ms4 * 1e-3), "ms_per_step": ms4,
                  "candidates": per4[-1]["candidates"], "junctions": per4[-1]["junctions"],
                  "tuned": cfg4,
                  "kernel_ms": {n: sum(x["ms_" + n] for x in per4) / len(per4)
                                for n in ("fill", "query", "record", "decide", "compact")}}
        log("long k %s" % long_k)
        p4.close()

    compare = None
    if args.compare:
        other = "standard" if args.filter == "blocked" else "blocked"
        p2 = plan_for(other)
        ms2, per2 = run_steps(p2, d_in, max(3, args.steps // 2), 1, stream)
        compare = {"filter": other, "value": bases / 1e9 / (ms2 * 1e-3), "ms_per_step": ms2,
                   "candidates": per2[-1]["candidates"], "junctions": per2[-1]["junctions"],
                   "kernel_ms": {n: sum(s["ms_" + n] for s in per2) / len(per2)
                                 for n in ("fill", "query", "record", "decide", "compact")}}
        log("compare %s" % compare)
        p2.close()

    primate = primate_leg(args, stream, tuned) if args.primate else None
    batched = batched_leg(args, stream) if args.sets > 0 else None
    serving = None
    if args.requests > 0:
        cap = batched["batched_gbps"] if batched else bases / 1e9 / (ms_per_step * 1e-3)
        serving = serving_leg(args, cap)

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(codes, k, b, h, args.cpu_sample, args.filter == "blocked")
        log("cpu baseline %s" % cpu)

    traffic, traffic_raw = measured_traffic(dom, args.filter, k)
    line = {
        "metric": "input Gbp/s for junction finding (pass1+pass2)",
        "value": bases / 1e9 / (ms_per_step * 1e-3),
        "unit": "Gbp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "%d bacterial genomes x 5 Mbp, k=%d, b=2^%d, h=%d, %s filter"
                               % (len(codes), k, args.bloom_log2, h, args.filter),
                   "input_mbp": round(bases / 1e6, 3), "k": k, "bloom_bits": b, "hashes": h,
                   "filter": args.filter},
        "pass12_gbps": bases / 1e9 / ((avg("ms_pass1") + avg("ms_pass2")) * 1e-3),
        "host_to_host": host,
        "kernel_ms": kernel_ms,
        "tuned": tuned,
        "counts": {n: st[n] for n in ("positions", "candidates", "junctions", "edges",
                                      "table_keys", "table_capacity", "query_probes",
                                      "fill_atomics", "table_probes")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_unscaled": traffic_raw,
                     "algorithmic_bytes": alg[dom], "granule": GRANULE,
                     "per_kernel_frac": {n: alg[n] / (kernel_ms[n] * 1e-3) / 1e9 / HBM_PEAK_GBS
                                         for n in kernel_ms}},
        "compare": compare,
        "rounds": rounds_leg,
        "long_k": long_k,
        "batched": batched,
        "serving": serving,
        "primate": primate,
        "cpu_baseline": cpu,
        "source_digest": source_digest(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
