// Host runtime behind the C ABI of twopaco.h: plan (layout of the genome
// set in HBM), validation, device buffers, the launch sequence of the two
// passes and the compaction, exact-table sizing and result download.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "layout.hpp"
#include "twopaco.h"

using namespace tp;

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(e_ == hipErrorOutOfMemory ? TP_ENOMEM : TP_EDEVICE,                \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                \
    } while (0)

namespace {

struct DevBuf {
    void *p = nullptr;
    uint64_t cap = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    // Grow to at least `bytes` (contents are not preserved).
    hipError_t ensure(uint64_t bytes) {
        if (bytes == 0)
            bytes = 16;
        bytes = (bytes + 255) & ~255ull;
        if (p && cap >= bytes)
            return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess)
            cap = bytes;
        else
            p = nullptr;
        return e;
    }
    template <class T> T *as() const { return (T *)p; }
};

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint64_t pow2_ceil(uint64_t x) {
    uint64_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

uint32_t log2_ceil(uint64_t x) {
    uint32_t l = 0;
    while ((1ull << l) < x)
        ++l;
    return l;
}

// HyperLogLog estimate (Flajolet et al. 2007) with the linear-counting
// correction for small cardinalities.
double hll_estimate(const uint32_t *reg) {
    const double m = HLL_M;
    double z = 0;
    uint32_t zeros = 0;
    for (uint32_t i = 0; i < HLL_M; ++i) {
        z += std::ldexp(1.0, -(int)reg[i]);
        zeros += reg[i] == 0;
    }
    double e = 0.7213 / (1 + 1.079 / m) * m * m / z;
    if (e <= 2.5 * m && zeros)
        e = m * std::log(m / zeros);
    return e;
}

}  // namespace

struct tp_plan {
    uint32_t n_genomes = 0, k = 0, h = 0, flags = 0;
    uint64_t b = 0;
    int W = 1;
    std::vector<uint64_t> n_bases, gbase;
    std::vector<DString> strings;
    uint64_t total = 0, n_tiles = 0, bitmap_words = 0, input_bytes = 0, positions = 0;
    uint32_t pf_log2 = 10;
    std::vector<uint32_t> tile_order;   // tiles grouped per XCD, slab by slab
    uint64_t xcd_start[NXCD + 1] = {};
    uint32_t grid[K_COUNT] = {};        // persistent grid per tile kernel

    int device = -1;
    bool static_uploaded = false;
    DevBuf d_tiles, d_strings, d_gbase, d_sent_raw, d_sent, d_pf, d_bloom, d_c1, d_j, d_cnt, d_hll;
    DevBuf d_keys, d_keys_hi, d_masks, d_blockcnt, d_blockoff;
    DevBuf d_pos, d_vertex, d_strand, d_sof, d_edges, d_joff;
    // run timeline: 0 start, 1 sentinels, 2 fill, 3 query, 4 pass 2 start,
    // 5 record start, 6 record end, 7 decide end, 8 compaction end
    hipEvent_t ev[9] = {};

    bool have_run = false;
    tp_stats stats{};
    uint64_t n_j = 0, n_e = 0;
    uint64_t *jbits = nullptr;  // J bitmap of the last run (C1 in pass-1-only mode)

    ~tp_plan() {
        for (auto &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};

static int validate_params(uint32_t k, uint64_t b, uint32_t h, uint32_t flags) {
    if (k < 1 || k > 63)
        return fail(TP_EINVAL, "k must be in 1..63");
    if (b < 32 || b > (1ull << 40) || (b & (b - 1)))
        return fail(TP_EINVAL, "bloom_bits must be a power of two in 2^5..2^40");
    if ((flags & TP_FLAG_BLOCKED_FILTER) && b < 64)
        return fail(TP_EINVAL, "the blocked filter needs bloom_bits >= 2^6");
    if (h < 1 || h > 16)
        return fail(TP_EINVAL, "hash_count must be in 1..16");
    if (flags & ~(TP_FLAG_SINGLE_STRAND | TP_FLAG_PASS1_ONLY | TP_FLAG_BLOCKED_FILTER))
        return fail(TP_EINVAL, "unknown flag bits");
    return TP_OK;
}

extern "C" const char *twopaco_last_error(void) { return g_err.c_str(); }

extern "C" int tp_plan_create(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                              uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                              tp_plan **out) {
    if (!out)
        return fail(TP_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_params(k, bloom_bits, hash_count, flags);
    if (rc)
        return rc;
    if (n_genomes && !genomes)
        return fail(TP_EINVAL, "genomes is NULL");
    tp_plan *p = new (std::nothrow) tp_plan;
    if (!p)
        return fail(TP_ENOMEM, "host allocation failed");
    p->n_genomes = n_genomes;
    p->k = k;
    p->h = hash_count;
    p->b = bloom_bits;
    p->flags = flags;
    p->W = k <= 31 ? 1 : 2;
    p->n_bases.resize(n_genomes);
    p->gbase.resize(n_genomes);
    uint64_t cursor = 0;
    for (uint32_t g = 0; g < n_genomes; ++g) {
        const tp_genome &G = genomes[g];
        if (G.n_nruns && !G.n_runs) {
            delete p;
            return fail(TP_EINVAL, "genome " + std::to_string(g) + ": n_runs is NULL");
        }
        p->n_bases[g] = G.n_bases;
        p->gbase[g] = cursor;
        // strings = complement of the N runs
        uint64_t prev_end = 0;
        for (uint64_t r = 0; r <= G.n_nruns; ++r) {
            uint64_t rs = r < G.n_nruns ? G.n_runs[2 * r] : G.n_bases;
            uint64_t rl = r < G.n_nruns ? G.n_runs[2 * r + 1] : 0;
            if (r < G.n_nruns &&
                (rl == 0 || rs < prev_end || rs > G.n_bases || rl > G.n_bases - rs)) {
                delete p;
                return fail(TP_EINVAL, "genome " + std::to_string(g) +
                                           ": N runs must be non-empty, sorted, disjoint and "
                                           "inside the genome");
            }
            if (rs - prev_end >= k) {
                DString s;
                s.gstart = cursor + prev_end;
                s.gend = cursor + rs;
                s.genome = g;
                s.pad = 0;
                p->strings.push_back(s);
                p->positions += rs - prev_end - k + 1;
            }
            prev_end = rs + rl;
        }
        cursor = align_up(cursor + G.n_bases, GENOME_ALIGN);
    }
    if (p->strings.size() >= (1ull << 31)) {
        delete p;
        return fail(TP_EINVAL, "too many strings");
    }
    p->total = align_up(cursor, TILE);
    p->n_tiles = p->total / TILE;
    if (p->n_tiles >= (1ull << 32)) {
        delete p;
        return fail(TP_EINVAL, "input too large");
    }
    // Slab s = tile s of every genome; slab s belongs to XCD s mod NXCD.
    {
        std::vector<uint64_t> first(n_genomes), count(n_genomes);
        uint64_t slabs = 0;
        for (uint32_t g = 0; g < n_genomes; ++g) {
            first[g] = p->gbase[g] / TILE;
            count[g] = (p->n_bases[g] + TILE - 1) / TILE;
            slabs = std::max(slabs, count[g]);
        }
        p->tile_order.reserve(p->n_tiles);
        for (uint32_t x = 0; x < NXCD; ++x) {
            p->xcd_start[x] = p->tile_order.size();
            for (uint64_t sl = x; sl < slabs; sl += NXCD)
                for (uint32_t g = 0; g < n_genomes; ++g)
                    if (sl < count[g])
                        p->tile_order.push_back((uint32_t)(first[g] + sl));
        }
        p->xcd_start[NXCD] = p->tile_order.size();
        if (p->tile_order.size() != p->n_tiles) {
            delete p;
            return fail(TP_EINVAL, "internal error: tile order does not cover the input");
        }
    }
    p->bitmap_words = p->total / 64;
    p->input_bytes = p->total / 4 + 64;
    p->pf_log2 = std::min<uint32_t>(PF_MAX_LOG2,
                                    std::max<uint32_t>(10, log2_ceil(2 * p->strings.size() * 32)));
    *out = p;
    return TP_OK;
}

extern "C" void tp_plan_destroy(tp_plan *p) { delete p; }

extern "C" uint64_t tp_plan_input_bytes(const tp_plan *p) { return p ? p->input_bytes : 0; }

extern "C" uint64_t tp_plan_genome_offset(const tp_plan *p, uint32_t g) {
    return (p && g < p->n_genomes) ? p->gbase[g] / 4 : 0;
}

extern "C" uint64_t tp_plan_bitmap_words(const tp_plan *p) { return p ? p->bitmap_words : 0; }

extern "C" uint64_t tp_plan_strings(const tp_plan *p) { return p ? p->strings.size() : 0; }

extern "C" int tp_plan_upload(tp_plan *p, const tp_genome *genomes, uint8_t *d_input,
                              void *stream) {
    if (!p || (!d_input && p->input_bytes))
        return fail(TP_EINVAL, "plan or device input is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemsetAsync(d_input, 0, p->input_bytes, s));
    for (uint32_t g = 0; g < p->n_genomes; ++g) {
        if (genomes[g].n_bases != p->n_bases[g])
            return fail(TP_EINVAL, "genome " + std::to_string(g) + " differs from the plan");
        if (!genomes[g].n_bases)
            continue;
        if (!genomes[g].packed)
            return fail(TP_EINVAL, "genome " + std::to_string(g) + ": packed is NULL");
        HIPCHK(hipMemcpyAsync(d_input + p->gbase[g] / 4, genomes[g].packed,
                              (genomes[g].n_bases + 3) / 4, hipMemcpyHostToDevice, s));
    }
    return TP_OK;
}

static SeqArgs seq_args(const tp_plan *p, const uint8_t *d_input) {
    SeqArgs a;
    a.seq = (const uint64_t *)d_input;
    a.seq_words = p->input_bytes / 8;
    a.strings = p->d_strings.as<DString>();
    a.n_strings = (uint32_t)p->strings.size();
    a.k = p->k;
    a.n_tiles = p->n_tiles;
    a.single = (p->flags & TP_FLAG_SINGLE_STRAND) ? 1u : 0u;
    a.pad = 0;
    a.tile_order = p->d_tiles.as<uint32_t>();
    for (uint32_t x = 0; x <= NXCD; ++x)
        a.xcd_start[x] = p->xcd_start[x];
    return a;
}

extern "C" int tp_run(tp_plan *p, const uint8_t *d_input, void *stream) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    if (!d_input && p->input_bytes)
        return fail(TP_EINVAL, "device input is NULL");
    if ((uintptr_t)d_input % 8)
        return fail(TP_EINVAL, "device input must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (p->device < 0)
        p->device = dev;
    else if (p->device != dev)
        return fail(TP_ESTATE, "plan is bound to another device");
    p->have_run = false;
    const uint64_t ns = p->strings.size();
    const int W = p->W;

    // ---- buffers that depend only on the plan
    HIPCHK(p->d_tiles.ensure(p->n_tiles * 4));
    HIPCHK(p->d_strings.ensure(ns * sizeof(DString)));
    HIPCHK(p->d_gbase.ensure((uint64_t)p->n_genomes * 8));
    HIPCHK(p->d_sent_raw.ensure(2 * ns * 8 * W));
    HIPCHK(p->d_sent.ensure(2 * ns * 8 * W));
    HIPCHK(p->d_pf.ensure((1ull << p->pf_log2) / 8));
    HIPCHK(p->d_bloom.ensure(p->b / 8));
    HIPCHK(p->d_c1.ensure(p->bitmap_words * 8));
    HIPCHK(p->d_cnt.ensure(sizeof(Counters)));
    HIPCHK(p->d_hll.ensure(HLL_M * 4));
    if (!p->static_uploaded) {
        if (p->n_tiles)
            HIPCHK(hipMemcpy(p->d_tiles.p, p->tile_order.data(), p->n_tiles * 4,
                             hipMemcpyHostToDevice));
        if (ns)
            HIPCHK(hipMemcpy(p->d_strings.p, p->strings.data(), ns * sizeof(DString),
                             hipMemcpyHostToDevice));
        if (p->n_genomes)
            HIPCHK(hipMemcpy(p->d_gbase.p, p->gbase.data(), (uint64_t)p->n_genomes * 8,
                             hipMemcpyHostToDevice));
        for (auto &e : p->ev)
            HIPCHK(hipEventCreate(&e));
        p->static_uploaded = true;
    }
    if (!p->grid[0]) {
        // persistent grids: every resident workgroup slot, a multiple of NXCD,
        // no more workgroups than tiles need
        int ncu = 0;
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        for (int kid = 0; kid < K_COUNT; ++kid) {
            int occ = 0;
            if (kid <= K_QUERY)
                HIPCHK(pass1_occupancy((KernelId)kid, W, (p->flags & TP_FLAG_BLOCKED_FILTER) != 0,
                                       &occ));
            else
                HIPCHK(pass2_occupancy((KernelId)kid, W, &occ));
            uint64_t g = (uint64_t)std::max(1, occ) * (uint64_t)std::max(1, ncu);
            g = std::min<uint64_t>(g, align_up(std::max<uint64_t>(p->n_tiles, 1), NXCD));
            p->grid[kid] = (uint32_t)std::max<uint64_t>(NXCD, g / NXCD * NXCD);
        }
    }
    const bool pass1_only = (p->flags & TP_FLAG_PASS1_ONLY) != 0;

    SeqArgs a = seq_args(p, d_input);
    BloomArgs f{p->d_bloom.as<uint32_t>(), p->b - 1, p->h,
                (p->flags & TP_FLAG_BLOCKED_FILTER) ? 1u : 0u};
    SentArgs sa{p->d_sent.p, (uint32_t)(2 * ns), p->pf_log2, p->d_pf.as<uint32_t>()};
    Counters *cnt = p->d_cnt.as<Counters>();
    Counters hc{};

    // ---- a0-a2: sentinels, first pass
    HIPCHK(hipEventRecord(p->ev[0], s));
    HIPCHK(launch_zero(cnt, sizeof(Counters), s));
    HIPCHK(launch_zero(p->d_hll.p, HLL_M * 4, s));
    HIPCHK(launch_zero(p->d_bloom.p, p->b / 8, s));
    HIPCHK(launch_sentinels(W, a, p->d_sent_raw.p, p->d_sent.p, p->d_pf.as<uint32_t>(),
                            p->pf_log2, s));
    HIPCHK(hipEventRecord(p->ev[1], s));
    HIPCHK(launch_fill(W, a, f, cnt, p->grid[K_FILL], s));
    HIPCHK(hipEventRecord(p->ev[2], s));
    HIPCHK(launch_query(W, a, f, sa, p->d_c1.as<uint64_t>(), cnt, p->d_hll.as<uint32_t>(),
                        p->grid[K_QUERY], s));
    HIPCHK(launch_popcount(f.words, p->b / 32, cnt, s));
    HIPCHK(hipEventRecord(p->ev[3], s));
    std::vector<uint32_t> hll(HLL_M);
    HIPCHK(hipMemcpyAsync(&hc, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hll.data(), p->d_hll.p, HLL_M * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    uint64_t cap = 0;
    uint32_t attempts = 0;
    double est = 0;
    HIPCHK(hipEventRecord(p->ev[4], s));
    if (pass1_only) {
        p->jbits = p->d_c1.as<uint64_t>();
        p->n_j = hc.candidates;
        for (int i = 5; i < 8; ++i)
            HIPCHK(hipEventRecord(p->ev[i], s));
    } else {
        // ---- a3-a4: second pass over the candidates
        HIPCHK(p->d_j.ensure(p->bitmap_words * 8));
        est = hll_estimate(hll.data());
        // load factor at most ~0.7 for the estimate (+15% for sketch error);
        // never more slots than twice the candidate count needs
        cap = pow2_ceil((uint64_t)std::ceil(est * 1.15 / 0.7));
        cap = std::min<uint64_t>(cap, pow2_ceil(2 * std::max<uint64_t>(hc.candidates, 1)));
        cap = std::max<uint64_t>(cap, 1024);
        for (;;) {
            ++attempts;
            TableArgs t;
            t.packed = p->k <= PACKED_MAX_K ? 1u : 0u;
            t.pad = 0;
            HIPCHK(p->d_keys.ensure(cap * 8));
            if (!t.packed)
                HIPCHK(p->d_masks.ensure(cap));
            if (W == 2)
                HIPCHK(p->d_keys_hi.ensure(cap * 8));
            t.keys = p->d_keys.as<unsigned long long>();
            t.keys_hi = W == 2 ? p->d_keys_hi.as<unsigned long long>() : nullptr;
            t.masks = t.packed ? nullptr : p->d_masks.as<uint32_t>();
            t.capmask = cap - 1;
            HIPCHK(launch_zero(&cnt->junctions, PASS2_COUNTERS * sizeof(unsigned long long), s));
            HIPCHK(launch_table_clear(W, t, s));
            HIPCHK(hipEventRecord(p->ev[5], s));
            HIPCHK(launch_record(W, a, p->d_c1.as<uint64_t>(), t, cnt, p->grid[K_RECORD], s));
            HIPCHK(hipEventRecord(p->ev[6], s));
            HIPCHK(launch_decide(W, a, sa, p->d_c1.as<uint64_t>(), t, p->d_j.as<uint64_t>(), cnt,
                                 p->grid[K_DECIDE], s));
            HIPCHK(hipEventRecord(p->ev[7], s));
            HIPCHK(hipMemcpyAsync(&hc, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (!hc.overflow)
                break;
            if (attempts >= 8 || cap >= (1ull << 40))
                return fail(TP_EOVERFLOW, "exact table overflowed after " +
                                              std::to_string(attempts) + " attempts");
            cap *= 2;
        }
        if (hc.missing)
            return fail(TP_EDEVICE, "internal error: " + std::to_string(hc.missing) +
                                        " candidate k-mers missing from the exact table");
        p->jbits = p->d_j.as<uint64_t>();
        p->n_j = hc.junctions;
    }

    // ---- a5: ordered compaction and edges
    const uint64_t nj = p->n_j;
    if (nj < ns)
        return fail(TP_EDEVICE, "internal error: fewer junctions than strings");
    const uint64_t ne = nj - ns;
    const uint64_t nblocks = (p->bitmap_words + SCAN_WORDS - 1) / SCAN_WORDS;
    HIPCHK(p->d_pos.ensure(nj * 8));
    HIPCHK(p->d_vertex.ensure(nj * 8 * W));
    HIPCHK(p->d_strand.ensure(nj));
    HIPCHK(p->d_sof.ensure(nj * 4));
    HIPCHK(p->d_edges.ensure(ne * sizeof(tp_edge)));
    HIPCHK(p->d_joff.ensure(((uint64_t)p->n_genomes + 1) * 8));
    HIPCHK(p->d_blockcnt.ensure(nblocks * 4));
    HIPCHK(p->d_blockoff.ensure((nblocks + 1) * 8));
    OutArgs o;
    o.pos = p->d_pos.as<uint64_t>();
    o.vertex = p->d_vertex.as<uint64_t>();
    o.strand = p->d_strand.as<uint8_t>();
    o.string_of = p->d_sof.as<uint32_t>();
    o.joff = p->d_joff.as<uint64_t>();
    o.edges = p->d_edges.p;
    o.gbase = p->d_gbase.as<uint64_t>();
    o.n_genomes = p->n_genomes;
    o.pad = 0;
    HIPCHK(launch_compact(W, a, p->jbits, p->bitmap_words, p->d_blockcnt.as<uint32_t>(),
                          p->d_blockoff.as<uint64_t>(), o, nj, s));
    HIPCHK(hipEventRecord(p->ev[8], s));
    HIPCHK(hipStreamSynchronize(s));

    tp_stats &st = p->stats;
    st = tp_stats{};
    st.positions = p->positions;
    st.candidates = hc.candidates;
    st.junctions = nj;
    st.edges = ne;
    st.bloom_popcount = hc.bloom_popcount;
    st.table_capacity = cap;
    st.table_keys = hc.table_keys;
    st.distinct_estimate = (uint64_t)est;
    st.table_attempts = attempts;
    st.sentinels = (uint32_t)(2 * ns);
    st.edge_positions = p->positions >= ns ? p->positions - ns : 0;
    st.fill_atomics = hc.fill_atomics;
    st.query_probes = hc.query_probes;
    st.table_probes = hc.table_probes;
    HIPCHK(hipEventElapsedTime(&st.ms_sentinels, p->ev[0], p->ev[1]));
    HIPCHK(hipEventElapsedTime(&st.ms_fill, p->ev[1], p->ev[2]));
    HIPCHK(hipEventElapsedTime(&st.ms_query, p->ev[2], p->ev[3]));
    HIPCHK(hipEventElapsedTime(&st.ms_record, p->ev[5], p->ev[6]));
    HIPCHK(hipEventElapsedTime(&st.ms_decide, p->ev[6], p->ev[7]));
    HIPCHK(hipEventElapsedTime(&st.ms_pass1, p->ev[0], p->ev[3]));
    HIPCHK(hipEventElapsedTime(&st.ms_pass2, p->ev[4], p->ev[7]));
    HIPCHK(hipEventElapsedTime(&st.ms_compact, p->ev[7], p->ev[8]));
    HIPCHK(hipEventElapsedTime(&st.ms_total, p->ev[0], p->ev[8]));
    p->n_e = ne;
    p->have_run = true;
    return TP_OK;
}

extern "C" int tp_get_stats(const tp_plan *p, tp_stats *out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    *out = p->stats;
    return TP_OK;
}

extern "C" int tp_get_device_outputs(const tp_plan *p, tp_device_outputs *out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    out->n_junctions = p->n_j;
    out->junction_offset = p->d_joff.as<uint64_t>();
    out->junction_pos = p->d_pos.as<uint64_t>();
    out->vertex = p->d_vertex.as<uint64_t>();
    out->strand = p->d_strand.as<uint8_t>();
    out->n_edges = p->n_e;
    out->edges = p->d_edges.as<tp_edge>();
    out->candidates = p->d_c1.as<uint64_t>();
    out->junction_bits = p->jbits;
    out->bloom = p->d_bloom.as<uint32_t>();
    return TP_OK;
}

// One host allocation holds the result header and all its arrays.
static tp_result *alloc_result(uint32_t n_genomes, uint64_t nj, uint64_t ne, int W) {
    uint64_t off_joff = align_up(sizeof(tp_result), 64);
    uint64_t off_pos = align_up(off_joff + ((uint64_t)n_genomes + 1) * 8, 64);
    uint64_t off_vx = align_up(off_pos + nj * 8, 64);
    uint64_t off_edges = align_up(off_vx + nj * 8 * W, 64);
    uint64_t off_strand = align_up(off_edges + ne * sizeof(tp_edge), 64);
    uint64_t total = off_strand + nj + 64;
    uint8_t *m = (uint8_t *)std::malloc(total);
    if (!m)
        return nullptr;
    tp_result *r = (tp_result *)m;
    std::memset(r, 0, sizeof(*r));
    r->junction_offset = (const uint64_t *)(m + off_joff);
    r->junction_pos = (const uint64_t *)(m + off_pos);
    r->vertex = (const uint64_t *)(m + off_vx);
    r->edges = (const tp_edge *)(m + off_edges);
    r->strand = (const uint8_t *)(m + off_strand);
    return r;
}

extern "C" int tp_download(const tp_plan *p, void *stream, tp_result **out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    *out = nullptr;
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    hipStream_t s = (hipStream_t)stream;
    tp_result *r = alloc_result(p->n_genomes, p->n_j, p->n_e, p->W);
    if (!r)
        return fail(TP_ENOMEM, "host allocation failed");
    r->n_genomes = p->n_genomes;
    r->kmer_words = (uint32_t)p->W;
    r->k = p->k;
    r->flags = p->flags;
    r->n_junctions = p->n_j;
    r->n_edges = p->n_e;
    r->stats = p->stats;
    auto cp = [&](const void *dst, const DevBuf &src, uint64_t bytes) -> hipError_t {
        if (!bytes)
            return hipSuccess;
        return hipMemcpyAsync((void *)dst, src.p, bytes, hipMemcpyDeviceToHost, s);
    };
    hipError_t e = cp(r->junction_offset, p->d_joff, ((uint64_t)p->n_genomes + 1) * 8);
    if (e == hipSuccess)
        e = cp(r->junction_pos, p->d_pos, p->n_j * 8);
    if (e == hipSuccess)
        e = cp(r->vertex, p->d_vertex, p->n_j * 8 * p->W);
    if (e == hipSuccess)
        e = cp(r->strand, p->d_strand, p->n_j);
    if (e == hipSuccess)
        e = cp(r->edges, p->d_edges, p->n_e * sizeof(tp_edge));
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        std::free(r);
        return fail(TP_EDEVICE, std::string("download: ") + hipGetErrorString(e));
    }
    *out = r;
    return TP_OK;
}

extern "C" void twopaco_result_free(tp_result *r) { std::free(r); }

extern "C" int tp_debug_bloom(const tp_plan *p, uint32_t *host_words, uint64_t n_words) {
    if (!p || !host_words)
        return fail(TP_EINVAL, "NULL argument");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    if (n_words != p->b / 32)
        return fail(TP_EINVAL, "n_words must be bloom_bits/32");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_words, p->d_bloom.p, n_words * 4, hipMemcpyDeviceToHost));
    return TP_OK;
}

extern "C" int tp_debug_candidates(const tp_plan *p, uint64_t *host_words, uint64_t n_words) {
    if (!p || !host_words)
        return fail(TP_EINVAL, "NULL argument");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    if (n_words != p->bitmap_words)
        return fail(TP_EINVAL, "n_words must be tp_plan_bitmap_words()");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_words, p->d_c1.p, n_words * 8, hipMemcpyDeviceToHost));
    return TP_OK;
}

extern "C" int twopaco_build_ex(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                                uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                                tp_result **out) {
    if (!out)
        return fail(TP_EINVAL, "out is NULL");
    *out = nullptr;
    tp_plan *p = nullptr;
    int rc = tp_plan_create(genomes, n_genomes, k, bloom_bits, hash_count, flags, &p);
    if (rc)
        return rc;
    uint8_t *d_input = nullptr;
    hipError_t e = hipMalloc(&d_input, std::max<uint64_t>(p->input_bytes, 16));
    if (e != hipSuccess) {
        tp_plan_destroy(p);
        return fail(e == hipErrorOutOfMemory ? TP_ENOMEM : TP_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    rc = tp_plan_upload(p, genomes, d_input, nullptr);
    if (!rc)
        rc = tp_run(p, d_input, nullptr);
    if (!rc)
        rc = tp_download(p, nullptr, out);
    (void)hipFree(d_input);
    tp_plan_destroy(p);
    return rc;
}

extern "C" int twopaco_build(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                             uint64_t bloom_bits, uint32_t hash_count, tp_result **out) {
    return twopaco_build_ex(genomes, n_genomes, k, bloom_bits, hash_count, 0, out);
}
