// The whole path on caller-owned device memory (tp_run_ws): a workspace and
// an output buffer laid out once per plan from stated bounds, so that a run
// is a plain sequence of kernel launches on the caller's stream -- no host
// wait, no allocation -- which a caller may capture in a HIP graph.
//
// Differences from tp_run, which sizes everything from counts it reads back:
//   - exact tables are sized from a bound on each set's distinct candidate
//     k-mers (a fraction of its positions) instead of the first pass's count
//     and sketch, and cannot grow: a set that overflows its table is flagged
//     in the status word instead of being rerun;
//   - outputs are sized for a bound on the junctions, and the compaction
//     writes at most that many (the junction offsets keep the true counts);
//   - with several rounds, the class partition runs on the device;
//   - counts are summed on the device into the output buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace tp;

namespace {

constexpr uint64_t WS_ALIGN = 256;

struct Carver {
    uint64_t at = 0;
    uint64_t take(uint64_t bytes) {
        const uint64_t o = at;
        at = align_up(at + std::max<uint64_t>(bytes, 1), WS_ALIGN);
        return o;
    }
};

static_assert(sizeof(tp_ws_counts) == 16 * 8, "tp_ws_counts is 16 words");
static_assert(sizeof(tp_ws_set_counters) == sizeof(SetCounters), "per-set counters");

}  // namespace

extern "C" int tp_plan_workspace_layout(tp_plan *p, double key_fraction, double junction_fraction,
                                        tp_ws_layout *out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    if (!(key_fraction > 0 && key_fraction <= 1) ||
        !(junction_fraction > 0 && junction_fraction <= 1))
        return fail(TP_EINVAL, "key_fraction and junction_fraction must be in (0, 1]");
    WsState w;
    const uint64_t ns = p->strings.size();
    const uint32_t nsets = (uint32_t)p->sets.size();
    const uint64_t ngen = p->n_bases.size();
    const uint64_t W = (uint64_t)p->W;
    const bool pass1_only = (p->flags & TP_FLAG_PASS1_ONLY) != 0;
    const uint32_t rounds = p->rounds;
    w.packed = table_packed(p);
    w.himask = table_himask(p);

    // exact tables for at most key_fraction x positions keys per set
    std::vector<double> keys(nsets);
    for (uint32_t i = 0; i < nsets; ++i)
        keys[i] = std::ceil(key_fraction * (double)p->sets[i].positions);
    std::vector<uint64_t> caps;
    if (!pass1_only) {
        caps = table_caps(p, keys, &w.pow2);
        w.desc = set_descs_for(p, caps, w.pow2, &w.slots);
    } else {
        caps.assign(nsets, 0);
        w.desc = set_descs_for(p, caps, true, &w.slots);
        w.slots = 0;
        for (auto &d : w.desc)
            d.table_off = d.table_m = d.table_e = 0;
    }
    w.bloom_starts.resize(nsets + 1);
    for (uint32_t i = 0; i < nsets; ++i)
        w.bloom_starts[i] = p->sets[i].bloom_off;
    w.bloom_starts[nsets] = p->bloom_words;
    w.nblocks = (p->bitmap_words + SCAN_WORDS - 1) / SCAN_WORDS;

    Carver c;
    w.o_tiles = c.take(p->n_tiles * 4);
    w.o_tile_info = c.take(p->n_tiles * sizeof(TileInfo));
    w.o_sets = c.take(nsets * sizeof(SetDesc));
    w.o_bloom_starts = c.take((nsets + 1) * 8ull);
    w.o_strings = c.take(ns * sizeof(DString));
    w.o_gbase = c.take(ngen * 8);
    w.o_sent_raw = c.take(2 * ns * 8 * W);
    w.o_sent = c.take(p->sent_tab_slots * 8 * W);
    w.o_sent_owner = c.take(p->sent_tab_slots * 4);
    w.o_pf = c.take((1ull << p->pf_log2) / 8);
    w.o_bloom = c.take(p->bloom_words * 4);
    w.o_c1 = c.take(p->bitmap_words * 8);
    w.o_c1u = rounds > 1 ? c.take(p->bitmap_words * 8) : w.o_c1;
    w.o_j = pass1_only ? w.o_c1u : c.take(p->bitmap_words * 8);
    w.o_cnt = c.take(sizeof(Counters));
    w.o_set_cnt = c.take(nsets * sizeof(SetCounters));
    w.o_census = rounds > 1 ? c.take((uint64_t)nsets * CLASS_Q * 8) : 0;
    w.o_bounds = rounds > 1 ? c.take((uint64_t)nsets * (rounds + 1) * 4) : 0;
    if (!pass1_only) {
        w.o_keys = c.take(w.slots * 8);
        w.o_keys_hi = W >= 2 ? c.take(w.slots * 8) : 0;
        w.o_keys_mid = W == 4 ? c.take(w.slots * 16) : 0;
        w.o_masks = (!w.packed && !w.himask) ? c.take(align_up(w.slots, 4)) : 0;
    }
    w.o_blockcnt = c.take(w.nblocks * 4);
    w.o_blockoff = c.take((w.nblocks + 1) * 8);
    w.o_queue = c.take(4 * NXCD * sizeof(unsigned int));  // tile queues of the tile kernels

    tp_ws_layout &L = w.pub;
    L = tp_ws_layout{};
    L.workspace_bytes = c.at;
    const uint64_t P = p->positions;
    L.max_junctions = std::max<uint64_t>(std::min<uint64_t>(
                                             P, (uint64_t)std::ceil(junction_fraction * (double)P)),
                                         std::min<uint64_t>(P, ns));
    L.max_edges = L.max_junctions;
    L.table_slots = w.slots;
    L.kmer_words = (uint32_t)W;
    L.rounds = rounds;
    Carver o;
    L.off_counts = o.take(sizeof(tp_ws_counts));
    L.off_joff = o.take((ngen + 1) * 8);
    L.off_pos = o.take(L.max_junctions * 8);
    L.off_vertex = o.take(L.max_junctions * 8 * W);
    L.off_strand = o.take(L.max_junctions);
    L.off_edges = o.take(L.max_edges * sizeof(tp_edge));
    L.output_bytes = o.at;
    L.ws_off_candidates = w.o_c1u;
    L.ws_off_junction_bits = w.o_j;
    L.ws_off_bloom = w.o_bloom;
    L.ws_off_set_counters = w.o_set_cnt;
    w.valid = true;
    w.gen = p->layout_gen;
    p->ws = std::move(w);
    *out = p->ws.pub;
    return TP_OK;
}

extern "C" uint64_t tp_plan_workspace_bytes(const tp_plan *p) {
    return (p && p->ws.valid && p->ws.gen == p->layout_gen) ? p->ws.pub.workspace_bytes : 0;
}

namespace tp {

// Layout tables into a workspace (asynchronous copies from the plan's host
// vectors, which outlive them).
int ws_prepare(tp_plan *p, uint8_t *base, hipStream_t s) {
    WsState &w = p->ws;
    if (!w.valid || w.gen != p->layout_gen)
        return fail(TP_ESTATE, "the plan has no current workspace layout "
                               "(tp_plan_workspace_layout)");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (p->device < 0)
        p->device = dev;
    else if (p->device != dev)
        return fail(TP_ESTATE, "plan is bound to another device");
    const int rc = plan_grids(p, dev);
    if (rc)
        return rc;
    std::memcpy(w.grid, p->grid, sizeof(w.grid));
    auto put = [&](uint64_t off, const void *src, uint64_t bytes) {
        return bytes ? hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s)
                     : hipSuccess;
    };
    HIPCHK(put(w.o_tiles, p->tile_order.data(), p->n_tiles * 4));
    HIPCHK(put(w.o_tile_info, p->tile_info.data(), p->n_tiles * sizeof(TileInfo)));
    HIPCHK(put(w.o_sets, w.desc.data(), w.desc.size() * sizeof(SetDesc)));
    HIPCHK(put(w.o_bloom_starts, w.bloom_starts.data(), w.bloom_starts.size() * 8));
    HIPCHK(put(w.o_strings, p->strings.data(), p->strings.size() * sizeof(DString)));
    HIPCHK(put(w.o_gbase, p->gbase.data(), p->gbase.size() * 8));
    w.prepared = base;
    return TP_OK;
}

// The launch sequence of a run on a prepared workspace.
int ws_run(tp_plan *p, const uint8_t *d_input, uint8_t *base, uint8_t *outb, hipStream_t s) {
    const WsState &w = p->ws;
    if (!w.valid || w.gen != p->layout_gen || w.prepared != base)
        return fail(TP_ESTATE, "the workspace was not prepared for the plan's current layout "
                               "(tp_plan_workspace_layout, tp_plan_prepare_workspace)");
    if (!d_input && p->input_bytes)
        return fail(TP_EINVAL, "device input is NULL");
    if ((uintptr_t)d_input % 8 || (uintptr_t)base % 8 || (uintptr_t)outb % 8)
        return fail(TP_EINVAL, "device buffers must be 8-byte aligned");
    if (!outb)
        return fail(TP_EINVAL, "output buffer is NULL");
    const uint64_t ns = p->strings.size();
    const uint32_t nsets = (uint32_t)p->sets.size();
    const int W = p->W;
    const bool pass1_only = (p->flags & TP_FLAG_PASS1_ONLY) != 0;
    const uint32_t rounds = p->rounds;
    const tp_ws_layout &L = w.pub;

    SeqArgs a;
    a.seq = (const uint64_t *)d_input;
    a.seq_words = p->input_bytes / 8;
    a.strings = (const DString *)(base + w.o_strings);
    a.n_strings = (uint32_t)ns;
    a.k = p->k;
    a.n_tiles = p->n_tiles;
    a.single = (p->flags & TP_FLAG_SINGLE_STRAND) ? 1u : 0u;
    a.sketch = 0;
    a.tile_order = (const uint32_t *)(base + w.o_tiles);
    for (uint32_t x = 0; x <= NXCD; ++x)
        a.xcd_start[x] = p->xcd_start[x];
    a.tiles = (const TileInfo *)(base + w.o_tile_info);
    a.sets = (const SetDesc *)(base + w.o_sets);
    a.set_cnt = (SetCounters *)(base + w.o_set_cnt);
    a.n_sets = nsets;
    a.classes = rounds > 1 ? 1u : 0u;
    a.pass2_slabs = p->cfg.pass2_slabs;
    a.fill_dedup = p->cfg.fill_dedup;
    a.chunk = p->cfg.chunk_tiles;
    a.pad = 0;
    a.queue = nullptr;  // set per launch below (tp_config.tile_queue)

    BloomArgs pool{(uint32_t *)(base + w.o_bloom), 0, p->h,
                   (p->flags & TP_FLAG_BLOCKED_FILTER) ? 1u : 0u};
    uint32_t *pf = (uint32_t *)(base + w.o_pf);
    SentArgs sa{base + w.o_sent, (uint32_t)(2 * ns), p->pf_log2, pf};
    Counters *cnt = (Counters *)(base + w.o_cnt);
    SetCounters *scnt = (SetCounters *)(base + w.o_set_cnt);
    uint64_t *c1 = (uint64_t *)(base + w.o_c1);
    uint64_t *c1u = rounds > 1 ? (uint64_t *)(base + w.o_c1u) : nullptr;
    uint64_t *jbits = (uint64_t *)(base + w.o_j);

    TableArgs t{};
    t.packed = w.packed ? 1u : 0u;
    t.himask = w.himask ? 1u : 0u;
    t.pow2 = w.pow2 ? 1u : 0u;
    t.keys = (unsigned long long *)(base + w.o_keys);
    t.keys_hi = W >= 2 ? (unsigned long long *)(base + w.o_keys_hi) : nullptr;
    t.keys_mid = W == 4 ? (unsigned long long *)(base + w.o_keys_mid) : nullptr;
    t.masks = (w.packed || w.himask) ? nullptr : (uint32_t *)(base + w.o_masks);

    // tile queues (tp_config.tile_queue): NXCD counters per tile kernel
    unsigned int *qbase = p->cfg.tile_queue ? (unsigned int *)(base + w.o_queue) : nullptr;
    auto queued = [&](int kid) { return with_queue(a, qbase, kid, w.grid[kid]); };
    // counters start at zero and add up over rounds; a set whose table
    // overflows keeps its flag, so its later rounds are skipped too
    HIPCHK(launch_zero(cnt, sizeof(Counters), s));
    HIPCHK(launch_zero(scnt, nsets * sizeof(SetCounters), s));
    HIPCHK(launch_sentinels(W, a, base + w.o_sent_raw, base + w.o_sent,
                            (uint32_t *)(base + w.o_sent_owner), p->sent_tab_slots, pf,
                            p->pf_log2, s));
    if (rounds > 1) {
        auto *census = (unsigned long long *)(base + w.o_census);
        auto *bounds = (uint32_t *)(base + w.o_bounds);
        HIPCHK(launch_census(W, a, census, w.grid[K_FILL], s));
        HIPCHK(launch_partition(census, nsets, rounds, bounds, s));
    }
    for (uint32_t round = 0; round < rounds; ++round) {
        if (rounds > 1)
            HIPCHK(launch_set_round((SetDesc *)(base + w.o_sets),
                                    (const uint32_t *)(base + w.o_bounds), nsets, rounds, round, s));
        HIPCHK(launch_zero(pool.words, p->bloom_words * 4, s));
        if (qbase)  // every tile kernel's queue, cleared by a kernel (graph-safe)
            HIPCHK(launch_zero(qbase, 4 * NXCD * sizeof(unsigned int), s));
        HIPCHK(launch_fill(W, queued(K_FILL), pool, cnt, w.grid[K_FILL], s));
        HIPCHK(launch_query(W, queued(K_QUERY), pool, sa, c1, c1u, round, cnt, nullptr,
                            w.grid[K_QUERY], s));
        HIPCHK(launch_popcount(pool.words, p->bloom_words, (const uint64_t *)(base + w.o_bloom_starts),
                               nsets, scnt, s));
        if (pass1_only)
            continue;
        HIPCHK(launch_table_clear(W, t, w.slots, s));
        HIPCHK(launch_record(W, queued(K_RECORD), c1, t, cnt, w.grid[K_RECORD], s));
        HIPCHK(launch_decide(W, queued(K_DECIDE), sa, c1, t, jbits, round > 0, cnt,
                             w.grid[K_DECIDE], s));
    }
    // pass-1-only: the candidates (their union over rounds) are the junctions
    const uint64_t *jb = pass1_only ? (rounds > 1 ? c1u : c1) : jbits;
    OutArgs o;
    o.pos = (uint64_t *)(outb + L.off_pos);
    o.vertex = (uint64_t *)(outb + L.off_vertex);
    o.strand = outb + L.off_strand;
    o.joff = (uint64_t *)(outb + L.off_joff);
    o.edges = outb + L.off_edges;
    o.gbase = (const uint64_t *)(base + w.o_gbase);
    o.n_genomes = (uint32_t)p->n_bases.size();
    o.pad = 0;
    HIPCHK(launch_compact_bound(W, a, jb, p->bitmap_words, (uint32_t *)(base + w.o_blockcnt),
                                (uint64_t *)(base + w.o_blockoff), o, L.max_junctions,
                                L.max_edges, s));
    FinalizeArgs f;
    f.set_cnt = scnt;
    f.cnt = cnt;
    f.blockoff = (const uint64_t *)(base + w.o_blockoff);
    f.nblocks = p->bitmap_words ? w.nblocks : 0;
    f.n_sets = nsets;
    f.pass2 = pass1_only ? 0u : 1u;
    f.n_strings = ns;
    f.positions = p->positions;
    f.max_j = L.max_junctions;
    f.out = (unsigned long long *)(outb + L.off_counts);
    HIPCHK(launch_ws_finalize(f, s));
    return TP_OK;
}

}  // namespace tp

extern "C" int tp_plan_prepare_workspace(tp_plan *p, void *d_workspace, void *stream) {
    if (!p || !d_workspace)
        return fail(TP_EINVAL, "NULL argument");
    if ((uintptr_t)d_workspace % WS_ALIGN)
        return fail(TP_EINVAL, "the workspace must be 256-byte aligned");
    return ws_prepare(p, (uint8_t *)d_workspace, (hipStream_t)stream);
}

extern "C" int tp_run_ws(tp_plan *p, const uint8_t *d_input, void *d_workspace, void *d_outputs,
                         void *stream) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    return ws_run(p, d_input, (uint8_t *)d_workspace, (uint8_t *)d_outputs, (hipStream_t)stream);
}
