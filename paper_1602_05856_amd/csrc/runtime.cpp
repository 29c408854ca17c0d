// Host runtime behind the C ABI of twopaco.h: plans (the layout of one or
// more genome sets in HBM), validation, device buffers, the launch sequence
// of the two passes and the compaction, exact-table sizing and result
// download.  A plain build is a batch of one set: every tile kernel reads its
// tile's set descriptor, so one launch per phase covers every set of a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <new>
#include <string>
#include <vector>

#include "hostmem.hpp"
#include "runtime.hpp"

using namespace tp;

static thread_local std::string g_err;

int tp::fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

namespace {

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

// Grow b to `bytes`; when the device is out of memory, free the buffers in
// `spare` (dead at that point of a run) and try once more.
static hipError_t ensure_spare(DevBuf &b, uint64_t bytes, std::initializer_list<DevBuf *> spare) {
    hipError_t e = b.ensure(bytes);
    if (e != hipErrorOutOfMemory)
        return e;
    (void)hipGetLastError();  // the failed allocation's error is not kept
    for (DevBuf *d : spare)
        d->release();
    return b.ensure(bytes);
}

// The compaction kernel writes edges as three 64-bit words.
static_assert(sizeof(tp_edge) == 24 && offsetof(tp_edge, from_pos) == 8 &&
                  offsetof(tp_edge, to_pos) == 16,
              "tp_edge layout");

tp_config tp::default_config(uint32_t n_sets) {
    tp_config c;
    // fill and query: all that fit; record and decision: 6 (more resident
    // workgroups only add contention on the table on every workload measured)
    c.wg_per_cu[K_FILL] = c.wg_per_cu[K_QUERY] = 0;
    c.wg_per_cu[K_RECORD] = c.wg_per_cu[K_DECIDE] = 6;
    c.tile_order = 0;
    c.table_load = n_sets == 1 ? 0.7f : 0.5f;
    c.graphs = 0;
    c.pass2_slabs = 2;  // decision in first-pass order, record in memory order
    c.fill_dedup = 1;
    c.table_shape = 0;
    c.chunk_tiles = 1;
    c.fill_binned = 0;
    c.bin_chunk_tiles = 0;
    c.bloom_bits_per_edge = 0;
    c.tile_queue = 1;
    c.record_binned = 0;
    c.record_passes = 0;
    c.reserved = 0;
    c.table_budget = 0;
    return c;
}

void tp::build_tile_order(tp_plan *p) {
    p->tile_order.clear();
    p->tile_order.reserve(p->n_tiles);
    if (p->cfg.tile_order == 1) {
        // memory order, cut in NXCD contiguous ranges
        for (uint32_t x = 0; x <= NXCD; ++x)
            p->xcd_start[x] = p->n_tiles * x / NXCD;
        for (uint64_t t = 0; t < p->n_tiles; ++t)
            p->tile_order.push_back((uint32_t)t);
        return;
    }
    // Slab j of a set = tile j of each of its genomes (homologous regions of
    // related genomes, which share filter lines).  Each XCD walks its slabs
    // set by set, so the workgroups running at one time probe one or two
    // sets' filters, not the whole pool.  Slabs go to XCDs round-robin,
    // continuing from set to set.
    std::vector<std::vector<uint32_t>> per_xcd(NXCD);
    uint64_t rr = 0;
    for (const SetInfo &si : p->sets) {
        uint64_t slabs = 0;
        for (uint32_t g = si.genome_lo; g < si.genome_hi; ++g)
            slabs = std::max<uint64_t>(slabs, (p->n_bases[g] + TILE - 1) / TILE);
        for (uint64_t sl = 0; sl < slabs; ++sl, ++rr)
            for (uint32_t g = si.genome_lo; g < si.genome_hi; ++g)
                if (sl * TILE < p->n_bases[g])
                    per_xcd[rr % NXCD].push_back((uint32_t)(p->gbase[g] / TILE + sl));
    }
    for (uint32_t x = 0; x < NXCD; ++x) {
        p->xcd_start[x] = p->tile_order.size();
        p->tile_order.insert(p->tile_order.end(), per_xcd[x].begin(), per_xcd[x].end());
    }
    // tiles of no genome (none today: genomes start on tile boundaries and
    // the input ends on one) still need an owner
    std::vector<uint8_t> seen(p->n_tiles, 0);
    for (uint32_t t : p->tile_order)
        seen[t] = 1;
    for (uint64_t t = 0; t < p->n_tiles; ++t)
        if (!seen[t])
            p->tile_order.push_back((uint32_t)t);
    p->xcd_start[NXCD] = p->tile_order.size();
}

static int validate_params(uint32_t k, uint32_t h, uint32_t flags) {
    if (k < 1 || k > 127)
        return fail(TP_EINVAL, "k must be in 1..127");
    if (h < 1 || h > 16)
        return fail(TP_EINVAL, "hash_count must be in 1..16");
    if (flags & ~(TP_FLAG_SINGLE_STRAND | TP_FLAG_PASS1_ONLY | TP_FLAG_BLOCKED_FILTER))
        return fail(TP_EINVAL, "unknown flag bits");
    return TP_OK;
}

static int validate_bloom(uint64_t b, uint32_t flags) {
    if (b < 32 || b > (1ull << 40) || (b & (b - 1)))
        return fail(TP_EINVAL, "bloom_bits must be a power of two in 2^5..2^40");
    if ((flags & TP_FLAG_BLOCKED_FILTER) && b < 64)
        return fail(TP_EINVAL, "the blocked filter needs bloom_bits >= 2^6");
    return TP_OK;
}

extern "C" const char *twopaco_last_error(void) { return g_err.c_str(); }

void tp::plan_clear_layout(tp_plan *p) {
    p->drop_graphs();
    p->k = p->h = p->flags = 0;
    p->W = 1;
    p->sets.clear();
    p->n_bases.clear();
    p->gbase.clear();
    p->strings.clear();
    p->tile_order.clear();
    p->tile_info.clear();
    for (auto &x : p->xcd_start)
        x = 0;
    p->total = p->n_tiles = p->bitmap_words = p->input_bytes = p->positions = 0;
    p->bloom_words = 0;
    p->sent_tab_slots = 0;
    p->pf_log2 = 10;
    for (auto &g : p->grid)
        g = 0;
    p->static_uploaded = p->order_uploaded = false;
    p->have_run = false;
    p->set_cnt.clear();
    p->joff.clear();
    p->n_j = p->n_e = 0;
    p->jbits = nullptr;
    p->c1_out = nullptr;
    p->rounds = 1;
    p->last_cap.clear();
    p->last_off.clear();
    p->table_live = false;
    ++p->layout_gen;
    p->ws = WsState{};
}

int tp::plan_layout(tp_plan *p, const tp_set *sets, uint32_t n_sets, uint32_t k,
                    uint32_t hash_count, uint32_t flags) {
    int rc = validate_params(k, hash_count, flags);
    if (rc)
        return rc;
    if (n_sets == 0)
        return fail(TP_EINVAL, "a batch needs at least one set");
    if (!sets)
        return fail(TP_EINVAL, "sets is NULL");
    uint64_t n_genomes = 0;
    for (uint32_t s = 0; s < n_sets; ++s) {
        if (sets[s].bloom_bits && (rc = validate_bloom(sets[s].bloom_bits, flags)))
            return fail(rc, "set " + std::to_string(s) + ": " + g_err);
        if (sets[s].n_genomes && !sets[s].genomes)
            return fail(TP_EINVAL, "set " + std::to_string(s) + ": genomes is NULL");
        n_genomes += sets[s].n_genomes;
    }
    if (n_genomes >= (1ull << 31))
        return fail(TP_EINVAL, "too many genomes");
    plan_clear_layout(p);
    p->k = k;
    p->h = hash_count;
    p->flags = flags;
    p->W = k <= 31 ? 1 : (k <= 63 ? 2 : 4);
    p->sets.resize(n_sets);
    uint64_t cursor = 0;
    for (uint32_t s = 0; s < n_sets; ++s) {
        SetInfo &si = p->sets[s];
        si.genome_lo = (uint32_t)p->n_bases.size();
        si.str_lo = (uint32_t)p->strings.size();
        si.b = sets[s].bloom_bits;
        si.b_auto = si.b == 0;
        for (uint32_t gi = 0; gi < sets[s].n_genomes; ++gi) {
            const tp_genome &G = sets[s].genomes[gi];
            const uint32_t g = (uint32_t)p->n_bases.size();
            const std::string where =
                n_sets == 1 ? "genome " + std::to_string(gi)
                            : "set " + std::to_string(s) + " genome " + std::to_string(gi);
            if (G.n_nruns && !G.n_runs) {
                plan_clear_layout(p);
                return fail(TP_EINVAL, where + ": n_runs is NULL");
            }
            p->n_bases.push_back(G.n_bases);
            p->gbase.push_back(cursor);
            // strings = complement of the N runs
            uint64_t prev_end = 0;
            for (uint64_t r = 0; r <= G.n_nruns; ++r) {
                uint64_t rs = r < G.n_nruns ? G.n_runs[2 * r] : G.n_bases;
                uint64_t rl = r < G.n_nruns ? G.n_runs[2 * r + 1] : 0;
                if (r < G.n_nruns &&
                    (rl == 0 || rs < prev_end || rs > G.n_bases || rl > G.n_bases - rs)) {
                    plan_clear_layout(p);
                    return fail(TP_EINVAL, where + ": N runs must be non-empty, sorted, "
                                                   "disjoint and inside the genome");
                }
                if (rs - prev_end >= k) {
                    DString d;
                    d.gstart = cursor + prev_end;
                    d.gend = cursor + rs;
                    d.genome = g;
                    d.set = s;
                    p->strings.push_back(d);
                    si.positions += rs - prev_end - k + 1;
                }
                prev_end = rs + rl;
            }
            cursor = align_up(cursor + G.n_bases, GENOME_ALIGN);
        }
        si.genome_hi = (uint32_t)p->n_bases.size();
        si.str_hi = (uint32_t)p->strings.size();
        p->positions += si.positions;
        // sentinel table: at most half full (2 sentinels per string)
        const uint64_t ns_set = 2ull * (si.str_hi - si.str_lo);
        si.sent_tab_off = p->sent_tab_slots;
        si.sent_tab_log2 = 0;
        if (ns_set) {
            si.sent_tab_log2 = std::max<uint32_t>(SENT_TAB_MIN_LOG2, log2_ceil(2 * ns_set));
            p->sent_tab_slots += 1ull << si.sent_tab_log2;
        }
    }
    if (p->strings.size() >= (1ull << 30)) {
        plan_clear_layout(p);
        return fail(TP_EINVAL, "too many strings");
    }
    p->total = align_up(cursor, TILE);
    p->n_tiles = p->total / TILE;
    if (p->n_tiles >= (1ull << 32)) {
        plan_clear_layout(p);
        return fail(TP_EINVAL, "input too large");
    }
    p->bitmap_words = p->total / 64;
    p->input_bytes = p->total / 4 + 64;
    p->pf_log2 = std::min<uint32_t>(PF_MAX_LOG2,
                                    std::max<uint32_t>(10, log2_ceil(2 * p->strings.size() * 32)));
    // Per-tile set and strings.  Strings are sorted and disjoint, so the
    // first string ending after a tile's start only moves forward.
    const uint32_t nstr = (uint32_t)p->strings.size();
    p->tile_info.assign(p->n_tiles, TileInfo{0, 0, 0, 0});
    for (uint32_t s = 0; s < n_sets; ++s)
        for (uint32_t g = p->sets[s].genome_lo; g < p->sets[s].genome_hi; ++g)
            for (uint64_t t = p->gbase[g] / TILE; t * TILE < p->gbase[g] + p->n_bases[g]; ++t)
                p->tile_info[t].set = s;
    for (uint64_t t = 0, lo = 0; t < p->n_tiles; ++t) {
        const uint64_t t0 = t * TILE, t1 = t0 + TILE;
        while (lo < nstr && p->strings[lo].gend <= t0)
            ++lo;
        uint64_t hi = lo;
        while (hi < nstr && p->strings[hi].gstart < t1)
            ++hi;
        p->tile_info[t].str_lo = (uint32_t)lo;
        p->tile_info[t].str_hi = (uint32_t)hi;
    }
    p->cfg = default_config(n_sets);
    layout_filters(p);
    build_tile_order(p);
    if (p->tile_order.size() != p->n_tiles) {
        plan_clear_layout(p);
        return fail(TP_EINVAL, "internal error: tile order does not cover the input");
    }
    return TP_OK;
}

// Smallest power of two >= bits_per_edge * edges, in 2^6..2^40.
static uint64_t bloom_bits_at(double bits_per_edge, uint64_t edges) {
    const double want = std::ceil(bits_per_edge * (double)edges);
    uint64_t b = 64;
    while (b < (1ull << 40) && (double)b < want)
        b <<= 1;
    return b;
}

void tp::layout_filters(tp_plan *p) {
    const uint32_t bpe = p->cfg.bloom_bits_per_edge ? p->cfg.bloom_bits_per_edge : 16;
    uint64_t bloom = 0;
    for (auto &si : p->sets) {
        if (si.b_auto) {
            // (k+1)-mer positions: one fewer than the k-mer positions per string
            const uint64_t nstr = si.str_hi - si.str_lo;
            si.b = bloom_bits_at(bpe, si.positions >= nstr ? si.positions - nstr : 0);
        }
        si.bloom_off = bloom;
        bloom = align_up(bloom + si.b / 32, BLOOM_ALIGN_WORDS);
    }
    p->bloom_words = bloom;
}

extern "C" uint64_t tp_bloom_bits_for(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                                     double bits_per_edge) {
    if ((n_genomes && !genomes) || k < 1 || !(bits_per_edge > 0))
        return 0;
    uint64_t edges = 0;  // (k+1)-mer positions: string length - k per string
    for (uint32_t g = 0; g < n_genomes; ++g) {
        const tp_genome &G = genomes[g];
        uint64_t prev_end = 0;
        for (uint64_t r = 0; r <= G.n_nruns; ++r) {
            uint64_t rs = r < G.n_nruns ? G.n_runs[2 * r] : G.n_bases;
            uint64_t rl = r < G.n_nruns ? G.n_runs[2 * r + 1] : 0;
            if (rs < prev_end || rs > G.n_bases)
                return 0;
            if (rs - prev_end > k)
                edges += rs - prev_end - k;
            prev_end = rs + rl;
        }
    }
    return bloom_bits_at(bits_per_edge, edges);
}


uint64_t tp::plan_device_bytes(const tp_plan *p) {
    uint64_t n = 0;
    const_cast<tp_plan *>(p)->for_each_buf([&](DevBuf &b) { n += b.cap; });
    return n;
}

void tp::plan_release(tp_plan *p) {
    p->drop_graphs();
    p->for_each_buf([](DevBuf &b) { b.release(); });
    p->static_uploaded = p->order_uploaded = false;
    p->have_run = false;
}

extern "C" int tp_batch_create(const tp_set *sets, uint32_t n_sets, uint32_t k,
                               uint32_t hash_count, uint32_t flags, tp_plan **out) {
    if (!out)
        return fail(TP_EINVAL, "out is NULL");
    *out = nullptr;
    tp_plan *p = new (std::nothrow) tp_plan;
    if (!p)
        return fail(TP_ENOMEM, "host allocation failed");
    const int rc = plan_layout(p, sets, n_sets, k, hash_count, flags);
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return TP_OK;
}

extern "C" int tp_plan_create(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                              uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                              tp_plan **out) {
    if (n_genomes && !genomes) {
        if (out)
            *out = nullptr;
        return fail(TP_EINVAL, "genomes is NULL");
    }
    tp_set one;
    one.genomes = genomes;
    one.n_genomes = n_genomes;
    one.reserved = 0;
    one.bloom_bits = bloom_bits;
    return tp_batch_create(&one, 1, k, hash_count, flags, out);
}

extern "C" void tp_plan_destroy(tp_plan *p) { delete p; }

extern "C" uint64_t tp_plan_input_bytes(const tp_plan *p) { return p ? p->input_bytes : 0; }

extern "C" uint64_t tp_plan_genome_offset(const tp_plan *p, uint32_t g) {
    return (p && g < p->n_bases.size()) ? p->gbase[g] / 4 : 0;
}

extern "C" uint64_t tp_plan_bitmap_words(const tp_plan *p) { return p ? p->bitmap_words : 0; }

extern "C" uint64_t tp_plan_strings(const tp_plan *p) { return p ? p->strings.size() : 0; }

extern "C" uint32_t tp_plan_sets(const tp_plan *p) { return p ? (uint32_t)p->sets.size() : 0; }

extern "C" uint32_t tp_plan_set_first_genome(const tp_plan *p, uint32_t set) {
    return (p && set < p->sets.size()) ? p->sets[set].genome_lo : 0;
}

extern "C" uint64_t tp_plan_set_bloom_offset(const tp_plan *p, uint32_t set) {
    return (p && set < p->sets.size()) ? p->sets[set].bloom_off : 0;
}

extern "C" uint64_t tp_plan_bloom_words(const tp_plan *p) { return p ? p->bloom_words : 0; }
extern "C" uint64_t tp_plan_set_bloom_bits(const tp_plan *p, uint32_t set) {
    return (p && set < p->sets.size()) ? p->sets[set].b : 0;
}

// Copy genomes, given as consecutive lists, to their places in the input.
static int upload_lists(tp_plan *p, const tp_genome *const *lists, const uint32_t *counts,
                        uint32_t n_lists, uint8_t *d_input, hipStream_t s) {
    if (!d_input && p->input_bytes)
        return fail(TP_EINVAL, "device input is NULL");
    HIPCHK(hipMemsetAsync(d_input, 0, p->input_bytes, s));
    uint32_t g = 0;
    for (uint32_t l = 0; l < n_lists; ++l) {
        if (counts[l] && !lists[l])
            return fail(TP_EINVAL, "genomes is NULL");
        for (uint32_t i = 0; i < counts[l]; ++i, ++g) {
            const tp_genome &G = lists[l][i];
            if (g >= p->n_bases.size() || G.n_bases != p->n_bases[g])
                return fail(TP_EINVAL, "genome " + std::to_string(g) + " differs from the plan");
            if (!G.n_bases)
                continue;
            if (!G.packed)
                return fail(TP_EINVAL, "genome " + std::to_string(g) + ": packed is NULL");
            HIPCHK(hipMemcpyAsync(d_input + p->gbase[g] / 4, G.packed, (G.n_bases + 3) / 4,
                                  hipMemcpyHostToDevice, s));
        }
    }
    if (g != p->n_bases.size())
        return fail(TP_EINVAL, "genome count differs from the plan");
    return TP_OK;
}

extern "C" int tp_plan_upload(tp_plan *p, const tp_genome *genomes, uint8_t *d_input,
                              void *stream) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    const uint32_t n = (uint32_t)p->n_bases.size();
    return upload_lists(p, &genomes, &n, 1, d_input, (hipStream_t)stream);
}

extern "C" int tp_batch_upload(tp_plan *p, const tp_set *sets, uint8_t *d_input, void *stream) {
    if (!p || !sets)
        return fail(TP_EINVAL, "plan or sets is NULL");
    const uint32_t ns = (uint32_t)p->sets.size();
    std::vector<const tp_genome *> lists(ns);
    std::vector<uint32_t> counts(ns);
    for (uint32_t s = 0; s < ns; ++s) {
        lists[s] = sets[s].genomes;
        counts[s] = sets[s].n_genomes;
        if (counts[s] != p->sets[s].genome_hi - p->sets[s].genome_lo)
            return fail(TP_EINVAL, "set " + std::to_string(s) + " differs from the plan");
    }
    return upload_lists(p, lists.data(), counts.data(), ns, d_input, (hipStream_t)stream);
}

// Greedy partition of the Multiple Rounds section: class c takes the longest
// run of consecutive subranges (at least one while any remain) whose counter
// sum times the number of classes stays within the total; the last class
// takes every remaining subrange.  bound[c] .. bound[c + 1] is class c.
void tp::class_partition(const uint64_t *e, uint32_t classes, uint32_t *bound) {
    unsigned __int128 total = 0;
    for (uint32_t i = 0; i < CLASS_Q; ++i)
        total += e[i];
    uint32_t next = 0;
    for (uint32_t c = 0; c < classes; ++c) {
        bound[c] = next;
        if (c + 1 == classes) {
            next = CLASS_Q;
            continue;
        }
        unsigned __int128 sum = 0;
        for (uint32_t taken = 0; next < CLASS_Q; ++taken, ++next) {
            if (taken > 0 && (sum + e[next]) * classes > total)
                break;
            sum += e[next];
        }
    }
    bound[classes] = CLASS_Q;
}

extern "C" int tp_plan_set_rounds(tp_plan *p, uint32_t rounds) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    if (rounds < 1 || rounds > MAX_ROUNDS)
        return fail(TP_EINVAL, "rounds must be in 1.." + std::to_string(MAX_ROUNDS));
    p->rounds = rounds;
    p->have_run = false;
    ++p->layout_gen;
    return TP_OK;
}

extern "C" uint32_t tp_plan_rounds(const tp_plan *p) { return p ? p->rounds : 0; }

extern "C" int tp_plan_class_bounds(const tp_plan *p, uint32_t set, uint32_t *bounds,
                                    uint32_t n) {
    if (!p || !bounds)
        return fail(TP_EINVAL, "NULL argument");
    if (set >= p->sets.size())
        return fail(TP_EINVAL, "set out of range");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    const uint32_t r = p->last_rounds;
    if (n != r + 1)
        return fail(TP_EINVAL, "n must be the last run's rounds + 1");
    if (r == 1) {
        bounds[0] = 0;
        bounds[1] = CLASS_Q;
        return TP_OK;
    }
    std::memcpy(bounds, &p->bounds[(size_t)set * (r + 1)], n * sizeof(uint32_t));
    return TP_OK;
}

extern "C" int tp_plan_get_config(const tp_plan *p, tp_config *out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    *out = p->cfg;
    return TP_OK;
}

extern "C" int tp_plan_set_config(tp_plan *p, const tp_config *cfg) {
    if (!p || !cfg)
        return fail(TP_EINVAL, "NULL argument");
    for (uint32_t w : cfg->wg_per_cu)
        if (w > 64)
            return fail(TP_EINVAL, "wg_per_cu must be 0 (all that fit) or 1..64");
    if (cfg->tile_order > 1)
        return fail(TP_EINVAL, "tile_order must be 0 or 1");
    if (!(cfg->table_load >= 0.05f && cfg->table_load <= 16.0f))
        return fail(TP_EINVAL, "table_load must be in [0.05, 16]");
    if (cfg->graphs > 1)
        return fail(TP_EINVAL, "graphs must be 0 or 1");
    if (cfg->pass2_slabs > 7)
        return fail(TP_EINVAL, "pass2_slabs must be in 0..7");
    if (cfg->fill_dedup > 1)
        return fail(TP_EINVAL, "fill_dedup must be 0 or 1");
    if (cfg->table_shape > 2)
        return fail(TP_EINVAL, "table_shape must be 0, 1 or 2");
    if (cfg->chunk_tiles < 1 || cfg->chunk_tiles > 64)
        return fail(TP_EINVAL, "chunk_tiles must be in 1..64");
    if (cfg->fill_binned > 2)
        return fail(TP_EINVAL, "fill_binned must be 0, 1 or 2");
    if (cfg->bin_chunk_tiles > BIN_CHUNK_TILES_MAX)
        return fail(TP_EINVAL, "bin_chunk_tiles must be 0 or 1.." +
                                   std::to_string(BIN_CHUNK_TILES_MAX));
    if (cfg->bloom_bits_per_edge > 256)
        return fail(TP_EINVAL, "bloom_bits_per_edge must be 0 (16) or 1..256");
    if (cfg->tile_queue > 1)
        return fail(TP_EINVAL, "tile_queue must be 0 or 1");
    if (cfg->record_binned > 2)
        return fail(TP_EINVAL, "record_binned must be 0, 1 or 2");
    if (cfg->record_passes > RBIN_MAX_PASSES)
        return fail(TP_EINVAL, "record_passes must be in 0.." + std::to_string(RBIN_MAX_PASSES));
    const bool reorder = cfg->tile_order != p->cfg.tile_order;
    const bool refilter = cfg->bloom_bits_per_edge != p->cfg.bloom_bits_per_edge;
    p->cfg = *cfg;
    if (refilter) {
        bool any_auto = false;
        for (const auto &si : p->sets)
            any_auto |= si.b_auto;
        if (any_auto) {
            layout_filters(p);
            p->static_uploaded = false;  // the set starts of the filter pool changed
        }
    }
    ++p->layout_gen;
    for (auto &g : p->grid)
        g = 0;
    if (reorder) {
        build_tile_order(p);
        p->order_uploaded = false;
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
    a.sketch = p->sets.size() == 1 ? 1u : 0u;
    a.tile_order = p->d_tiles.as<uint32_t>();
    for (uint32_t x = 0; x <= NXCD; ++x)
        a.xcd_start[x] = p->xcd_start[x];
    a.tiles = p->d_tile_info.as<TileInfo>();
    a.sets = p->d_sets.as<SetDesc>();
    a.set_cnt = p->d_set_cnt.as<SetCounters>();
    a.n_sets = (uint32_t)p->sets.size();
    a.classes = 0;
    a.pass2_slabs = p->cfg.pass2_slabs;
    a.fill_dedup = p->cfg.fill_dedup;
    a.chunk = p->cfg.chunk_tiles;
    a.pad = 0;
    a.queue = nullptr;
    return a;
}

// The sequence arguments of tile kernel kid, with its tile queue (NXCD
// counters at qbase + kid * NXCD) when queues are on and the kernel has at
// least QUEUE_MIN_TILES tiles per workgroup of its grid (with fewer, a
// claim's workgroup barriers cost more than balancing gains).
constexpr uint64_t QUEUE_MIN_TILES = 4;
SeqArgs tp::with_queue(SeqArgs a, unsigned int *qbase, int kid, uint32_t grid) {
    a.queue = qbase && a.n_tiles >= QUEUE_MIN_TILES * grid ? qbase + kid * NXCD : nullptr;
    return a;
}

// Set descriptors for the current table layout.
static std::vector<SetDesc> set_descs(const tp_plan *p) {
    std::vector<SetDesc> d(p->sets.size());
    for (size_t s = 0; s < p->sets.size(); ++s) {
        const SetInfo &si = p->sets[s];
        d[s].bloom_off = si.bloom_off;
        d[s].bloom_mask = si.b - 1;
        d[s].table_off = si.table_off;
        if (p->table_pow2) {
            d[s].table_m = 1;
            d[s].table_e = log2_ceil(si.table_cap);
        } else {
            (void)shape_table(si.table_cap, &d[s].table_m, &d[s].table_e);
        }
        d[s].sent_lo = 2 * si.str_lo;
        d[s].sent_hi = 2 * si.str_hi;
        d[s].sent_tab_off = si.sent_tab_off;
        d[s].sent_tab_log2 = si.sent_tab_log2;
        d[s].pad = 0;
        d[s].str_lo = si.str_lo;
        d[s].str_hi = si.str_hi;
    }
    return d;
}

bool tp::table_packed(const tp_plan *p) { return p->k <= PACKED_MAX_K; }

bool tp::table_himask(const tp_plan *p) {
    return p->W >= 2 && 2 * p->k <= 64 * (uint32_t)(p->W - 1) + HIMASK_SHIFT;
}

std::vector<uint64_t> tp::table_caps(const tp_plan *p, const std::vector<double> &keys,
                                     bool *pow2) {
    const size_t nsets = keys.size();
    const double load = p->cfg.table_load;
    const uint64_t slot_bytes =
        8ull * p->W + (table_packed(p) || table_himask(p) ? 0 : 1);
    std::vector<uint64_t> exact(nsets), caps(nsets);
    uint64_t waste = 0;
    for (size_t i = 0; i < nsets; ++i) {
        const double want = std::min(std::ceil(std::max(keys[i], 1.0) / load), (double)MAX_TABLE);
        exact[i] = std::max((uint64_t)want, MIN_TABLE);
        waste += (pow2_ceil(exact[i]) - exact[i]) * slot_bytes;
    }
    *pow2 = p->cfg.table_shape == 1 || (p->cfg.table_shape == 0 && waste <= POW2_WASTE_BYTES);
    for (size_t i = 0; i < nsets; ++i) {
        uint32_t m = 0, e = 0;
        caps[i] = *pow2 ? pow2_ceil(exact[i]) : shape_table(exact[i], &m, &e);
    }
    return caps;
}

std::vector<SetDesc> tp::set_descs_for(const tp_plan *p, const std::vector<uint64_t> &caps,
                                       bool pow2, uint64_t *slots) {
    std::vector<SetDesc> d(p->sets.size());
    uint64_t off = 0;
    for (size_t s = 0; s < p->sets.size(); ++s) {
        const SetInfo &si = p->sets[s];
        d[s].bloom_off = si.bloom_off;
        d[s].bloom_mask = si.b - 1;
        d[s].table_off = off;
        if (pow2) {
            d[s].table_m = 1;
            d[s].table_e = log2_ceil(caps[s]);
        } else {
            (void)shape_table(caps[s], &d[s].table_m, &d[s].table_e);
        }
        off += caps[s] + TABLE_TAIL;
        d[s].sent_lo = 2 * si.str_lo;
        d[s].sent_hi = 2 * si.str_hi;
        d[s].sent_tab_off = si.sent_tab_off;
        d[s].sent_tab_log2 = si.sent_tab_log2;
        d[s].pad = 0;
        d[s].str_lo = si.str_lo;
        d[s].str_hi = si.str_hi;
        d[s].cls_lo = d[s].cls_hi = 0;
    }
    *slots = off;
    return d;
}

int tp::plan_grids(tp_plan *p, int dev) {
    // persistent grids: the configured resident workgroups per CU (at most
    // what fits), a multiple of NXCD, no more than the tiles need
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (p->cu_limit)
        ncu = std::min<int>(ncu, (int)p->cu_limit);
    p->n_cu = (uint32_t)std::max(1, ncu);
    for (int kid = 0; kid < K_COUNT; ++kid) {
        int occ = 0;
        if (kid <= K_QUERY)
            HIPCHK(pass1_occupancy((KernelId)kid, p->W, (p->flags & TP_FLAG_BLOCKED_FILTER) != 0,
                                   p->cfg.fill_dedup != 0, &occ));
        else
            HIPCHK(pass2_occupancy((KernelId)kid, p->W, &occ));
        occ = std::max(1, occ);
        if (p->cfg.wg_per_cu[kid])
            occ = std::min<int>(occ, (int)p->cfg.wg_per_cu[kid]);
        uint64_t g = (uint64_t)occ * (uint64_t)std::max(1, ncu);
        g = std::min<uint64_t>(g, align_up(std::max<uint64_t>(p->n_tiles, 1), NXCD));
        p->grid[kid] = (uint32_t)std::max<uint64_t>(NXCD, g / NXCD * NXCD);
    }
    return TP_OK;
}

namespace {

// Bytes of every argument a launch sequence depends on.
struct KeyBuilder {
    std::vector<uint8_t> v;
    template <class T> KeyBuilder &operator()(const T &x) {
        const uint8_t *b = (const uint8_t *)&x;
        v.insert(v.end(), b, b + sizeof(T));
        return *this;
    }
};

// Enqueue a launch sequence on the run's stream, or (graphs on) replay its
// captured graph, capturing it first when none exists for these arguments.
template <class F>
int run_segment(tp_plan *p, bool graphs, int which, const std::vector<uint8_t> &key,
                hipStream_t s, F &&enqueue) {
    if (!graphs)
        return enqueue(s);
    Segment &g = p->seg[which];
    if (!g.exec || g.key != key) {
        if (g.exec)
            HIPCHK(hipGraphExecDestroy(g.exec));
        g.exec = nullptr;
        g.key.clear();
        if (!p->cap)
            HIPCHK(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue(p->cap);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(p->cap, &graph);
        if (rc) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rc;
        }
        HIPCHK(e);
        const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(ei);
        g.key = key;
    }
    HIPCHK(hipGraphLaunch(g.exec, s));
    return TP_OK;
}

}  // namespace

// Device bytes the plan will hold once each listed buffer has grown to at
// least its size (buffers only grow; the others keep their capacity).
static uint64_t bytes_after(tp_plan *p, std::initializer_list<std::pair<DevBuf *, uint64_t>> grow) {
    uint64_t n = plan_device_bytes(p);
    for (const auto &g : grow) {
        const uint64_t want = (std::max<uint64_t>(g.second, 16) + 255) & ~255ull;
        if (want > g.first->cap)
            n += want - g.first->cap;
    }
    return n;
}

// Ask the plan's owner (a server) for the device bytes a growth needs.
static int reserve(tp_plan *p, std::initializer_list<std::pair<DevBuf *, uint64_t>> grow) {
    if (!p->grow_hook)
        return TP_OK;
    return p->grow_hook(p->grow_ctx, bytes_after(p, grow));
}

constexpr int RUN_SPLIT = 1;  // run_impl: redo the run with *split rounds

constexpr uint64_t BIN_AUTO_BYTES = 1ull << 30;  // binned fill by default from this set filter size

// Whether this plan's fill can run binned: blocked filter, a pool within the
// bucket limit.
bool tp::fill_binnable(const tp_plan *p) {
    if (!(p->flags & TP_FLAG_BLOCKED_FILTER) || !p->n_tiles)
        return false;
    const uint64_t blocks = p->bloom_words / 2;
    const uint64_t per_bucket = (uint64_t)BIN_REGION * BIN_SUB;
    return (blocks + per_bucket - 1) / per_bucket <= BIN_MAX_BUCKETS;
}

// Whether this plan's fill runs binned (tp_config.fill_binned): by default
// when some set's own filter is 1 GiB or more (many small filters of a
// batch stay in the caches while their tiles run, and fill faster with
// atomics).
static bool fill_binned(const tp_plan *p) {
    if (p->cfg.fill_binned == 1 || !fill_binnable(p))
        return false;
    uint64_t largest = 0;
    for (const auto &si : p->sets)
        largest = std::max<uint64_t>(largest, si.b / 8);
    return p->cfg.fill_binned == 2 || largest >= BIN_AUTO_BYTES;
}

// The binned fill's scratch: items in the exact table's key buffer (dead
// during the first pass), counts and offsets in d_bin.  Sets *chunk_tiles.
static int bin_setup(tp_plan *p, BinArgs *b, uint32_t *chunk_tiles,
                     std::initializer_list<DevBuf *> outputs) {
    *b = BinArgs{};
    // default: 2^31 positions, or as many as the key buffer already holds
    // (a table from an earlier run) up to 2^33; fewer chunks reread the
    // filter fewer times
    uint64_t want = p->cfg.bin_chunk_tiles;
    if (!want)
        want = std::min<uint64_t>(4ull * BIN_CHUNK_TILES_MAX,
                                  std::max<uint64_t>(BIN_CHUNK_TILES_MAX,
                                                     p->d_keys.cap / (2 * 8 * TILE)));
    const uint64_t tiles = std::min<uint64_t>(p->n_tiles, want);
    *chunk_tiles = (uint32_t)tiles;
    const uint64_t items = tiles * TILE;
    b->n_blocks = p->bloom_words / 2;
    const uint64_t regions = (b->n_blocks + BIN_REGION - 1) / BIN_REGION;
    b->n_buckets = (uint32_t)((regions + BIN_SUB - 1) / BIN_SUB);
    b->grid = (uint32_t)std::min<uint64_t>((uint64_t)BIN_WG_PER_CU * std::max<uint32_t>(1, p->n_cu),
                                           tiles);
    const uint64_t n_counts = (uint64_t)b->n_buckets * b->grid;
    const uint64_t o_off = align_up(n_counts * 4, 256);
    const uint64_t o_reg = o_off + align_up((n_counts + 1) * 8, 256);
    const uint64_t meta = o_reg + ((uint64_t)b->n_buckets * BIN_SUB + 1) * 8;
    const int rc = reserve(p, {{&p->d_keys, 2 * items * 8}, {&p->d_bin, meta}});
    if (rc)
        return rc;
    HIPCHK(ensure_spare(p->d_keys, 2 * items * 8, outputs));
    HIPCHK(ensure_spare(p->d_bin, meta, outputs));
    b->items_a = p->d_keys.as<uint64_t>();
    b->items_b = b->items_a + items;
    uint8_t *m = p->d_bin.as<uint8_t>();
    b->counts = (uint32_t *)m;
    b->offsets = (uint64_t *)(m + o_off);
    b->region_off = (uint64_t *)(m + o_reg);
    return TP_OK;
}

constexpr uint32_t RBIN_AUTO_PASSES = 2;  // binned record by default: at most this many passes
constexpr uint64_t RBIN_MEM_MARGIN = 1ull << 30;  // device bytes left free by its own scratch

// The binned record's scratch (tp_config.record_binned) for a one-set plan
// with packed slots whose table has n_blocks home blocks: two arrays of
// rb->cap items, and the passes they take (the fewest found): in the last
// run's edge array (dead until the compaction), or in d_rbin, grown for
// record_passes passes (at least one) when the device has room.  By default
// at most RBIN_AUTO_PASSES passes (any number when forced).  *use = false:
// the record runs directly (also for plans of a server, which budgets their
// memory).
static int rbin_setup(tp_plan *p, uint64_t candidates, uint64_t n_blocks, uint64_t table_bytes,
                      RecBinArgs *rb, uint32_t *passes, bool *use) {
    *use = false;
    const uint32_t mode = p->cfg.record_binned;
    if (mode == 1 || (mode == 0 && table_bytes < BIN_AUTO_BYTES) || p->grow_hook)
        return TP_OK;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)BIN_WG_PER_CU * std::max<uint32_t>(1, p->n_cu),
                              p->n_tiles));
    const uint64_t slack = (uint64_t)grid * RBIN_SEG;  // partly filled staging segments
    const uint64_t want = (uint64_t)((double)candidates * 1.05) + 1;  // items, all passes
    const uint64_t per_max = (uint64_t)BIN_MAX_BUCKETS * BIN_SUB;     // blocks per pass
    const uint64_t min_passes = std::max<uint64_t>(
        {1, p->cfg.record_passes, (n_blocks + per_max - 1) / per_max});
    const uint64_t max_passes = mode == 2 ? RBIN_MAX_PASSES : RBIN_AUTO_PASSES;
    auto passes_for = [&](uint64_t bytes) -> uint64_t {  // 0: too small
        const uint64_t cap = bytes / 16;
        if (cap <= slack)
            return 0;
        const uint64_t n = std::max(min_passes, (want + cap - slack - 1) / (cap - slack));
        return n <= max_passes ? n : 0;
    };
    if (min_passes > max_passes)
        return TP_OK;
    // the fewest passes: the edge array, d_rbin as it is, or d_rbin grown
    // for min_passes when the device has room
    DevBuf *buf = nullptr;
    uint64_t n = 0;
    for (DevBuf *b : {&p->d_edges, &p->d_rbin}) {
        const uint64_t nb = passes_for(b->cap);
        if (nb && (!n || nb < n)) {
            n = nb;
            buf = b;
        }
    }
    if (!n || n > min_passes) {
        const uint64_t need = 16 * ((want + min_passes - 1) / min_passes + slack);
        size_t free_b = 0, total_b = 0;
        HIPCHK(hipMemGetInfo(&free_b, &total_b));
        if (need + RBIN_MEM_MARGIN <= free_b + p->d_rbin.cap) {
            if (p->d_rbin.ensure(need) == hipSuccess) {
                n = passes_for(p->d_rbin.cap);
                buf = &p->d_rbin;
            } else {
                (void)hipGetLastError();  // not kept: as found, or the record runs directly
                n = passes_for(p->d_edges.cap);
                buf = &p->d_edges;
            }
        }
    }
    if (!n)
        return TP_OK;
    const uint64_t per_pass = (n_blocks + n - 1) / n;
    n = (n_blocks + per_pass - 1) / per_pass;  // the passes the blocks take
    const uint64_t nbk = (per_pass + BIN_SUB - 1) / BIN_SUB;
    const uint64_t o_off = align_up(nbk * grid * 4, 256);
    const uint64_t o_reg = o_off + align_up((nbk * grid + 1) * 8, 256);
    const uint64_t o_ctl = o_reg + align_up((nbk * BIN_SUB + 1) * 8, 256);
    if (p->d_bin.ensure(o_ctl + 256) != hipSuccess) {
        (void)hipGetLastError();
        return TP_OK;
    }
    *rb = RecBinArgs{};
    rb->cap = buf->cap / 16;
    rb->items_a = buf->as<uint64_t>();
    rb->items_b = rb->items_a + rb->cap;
    uint8_t *m = p->d_bin.as<uint8_t>();
    rb->counts = (uint32_t *)m;
    rb->offsets = (uint64_t *)(m + o_off);
    rb->region_off = (uint64_t *)(m + o_reg);
    rb->ctl = (unsigned long long *)(m + o_ctl);
    rb->grid = grid;
    *passes = (uint32_t)n;
    *use = true;
    return TP_OK;
}

static int run_impl(tp_plan *p, const uint8_t *d_input, hipStream_t s, uint32_t rounds,
                    uint32_t *split);

extern "C" int tp_run(tp_plan *p, const uint8_t *d_input, void *stream) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    if (!d_input && p->input_bytes)
        return fail(TP_EINVAL, "device input is NULL");
    if ((uintptr_t)d_input % 8)
        return fail(TP_EINVAL, "device input must be 8-byte aligned");
    uint32_t split = 0;
    int rc = run_impl(p, d_input, (hipStream_t)stream, p->rounds, &split);
    if (rc == RUN_SPLIT)
        rc = run_impl(p, d_input, (hipStream_t)stream, split, nullptr);
    return rc;
}

static int run_impl(tp_plan *p, const uint8_t *d_input, hipStream_t s, uint32_t rounds,
                    uint32_t *split) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (p->device < 0)
        p->device = dev;
    else if (p->device != dev)
        return fail(TP_ESTATE, "plan is bound to another device");
    p->have_run = false;
    p->table_live = false;
    const uint64_t ns = p->strings.size();
    const uint32_t nsets = (uint32_t)p->sets.size();
    const uint64_t ngen = p->n_bases.size();
    const int W = p->W;

    // ---- buffers that depend only on the plan
    HIPCHK(p->d_tiles.ensure(p->n_tiles * 4));
    HIPCHK(p->d_tile_info.ensure(p->n_tiles * sizeof(TileInfo)));
    HIPCHK(p->d_sets.ensure(nsets * sizeof(SetDesc)));
    HIPCHK(p->d_bloom_starts.ensure((nsets + 1) * 8ull));
    HIPCHK(p->d_strings.ensure(ns * sizeof(DString)));
    HIPCHK(p->d_gbase.ensure(ngen * 8));
    HIPCHK(p->d_sent_raw.ensure(2 * ns * 8 * W));
    HIPCHK(p->d_sent.ensure(p->sent_tab_slots * 8 * W));
    HIPCHK(p->d_sent_owner.ensure(p->sent_tab_slots * 4));
    HIPCHK(p->d_pf.ensure((1ull << p->pf_log2) / 8));
    HIPCHK(p->d_bloom.ensure(p->bloom_words * 4));
    HIPCHK(p->d_c1.ensure(p->bitmap_words * 8));
    HIPCHK(p->d_cnt.ensure(sizeof(Counters)));
    HIPCHK(p->d_set_cnt.ensure(nsets * sizeof(SetCounters)));
    HIPCHK(p->d_hll.ensure(HLL_M * 4));
    HIPCHK(p->d_queue.ensure(4 * NXCD * sizeof(unsigned int)));
    // Layout tables go up on the run's own stream: a copy on the null
    // stream would also wait for the work of every other blocking stream of
    // the device (another server worker's job, say).  Their host copies are
    // the plan's and stay put until the next layout.
    if (!p->static_uploaded) {
        if (p->n_tiles)
            HIPCHK(hipMemcpyAsync(p->d_tile_info.p, p->tile_info.data(),
                                  p->n_tiles * sizeof(TileInfo), hipMemcpyHostToDevice, s));
        if (ns)
            HIPCHK(hipMemcpyAsync(p->d_strings.p, p->strings.data(), ns * sizeof(DString),
                                  hipMemcpyHostToDevice, s));
        if (ngen)
            HIPCHK(hipMemcpyAsync(p->d_gbase.p, p->gbase.data(), ngen * 8,
                                  hipMemcpyHostToDevice, s));
        p->bloom_starts.assign(nsets + 1, 0);
        for (uint32_t i = 0; i < nsets; ++i)
            p->bloom_starts[i] = p->sets[i].bloom_off;
        p->bloom_starts[nsets] = p->bloom_words;
        HIPCHK(hipMemcpyAsync(p->d_bloom_starts.p, p->bloom_starts.data(),
                              p->bloom_starts.size() * 8, hipMemcpyHostToDevice, s));
        for (auto &e : p->ev)
            if (!e)
                HIPCHK(hipEventCreate(&e));
        p->static_uploaded = true;
    }
    if (!p->order_uploaded) {
        if (p->n_tiles)
            HIPCHK(hipMemcpyAsync(p->d_tiles.p, p->tile_order.data(), p->n_tiles * 4,
                                  hipMemcpyHostToDevice, s));
        p->order_uploaded = true;
    }
    if (!p->grid[0]) {
        const int rcg = plan_grids(p, dev);
        if (rcg)
            return rcg;
    }
    const bool pass1_only = (p->flags & TP_FLAG_PASS1_ONLY) != 0;
    p->last_rounds = rounds;
    for (auto &si : p->sets)
        si.table_cap = si.table_off = 0;
    std::vector<SetDesc> desc = set_descs(p);

    SeqArgs a = seq_args(p, d_input);
    a.classes = rounds > 1 ? 1u : 0u;
    BloomArgs pool{p->d_bloom.as<uint32_t>(), 0, p->h,
                   (p->flags & TP_FLAG_BLOCKED_FILTER) ? 1u : 0u};
    SentArgs sa{p->d_sent.p, (uint32_t)(2 * ns), p->pf_log2, p->d_pf.as<uint32_t>()};
    const uint64_t sent_slots = p->sent_tab_slots;
    Counters *cnt = p->d_cnt.as<Counters>();
    SetCounters *scnt = p->d_set_cnt.as<SetCounters>();
    Counters hc{}, total_cnt{};
    std::vector<SetCounters> hs(nsets), tot(nsets);
    std::vector<uint64_t> max_cap(nsets, 0);
    uint64_t *c1u = nullptr;
    if (rounds > 1) {
        HIPCHK(p->d_c1u.ensure(p->bitmap_words * 8));
        c1u = p->d_c1u.as<uint64_t>();
    }
    p->c1_out = rounds > 1 ? c1u : p->d_c1.as<uint64_t>();

    // binned fill: its scratch (the previous run's outputs are dead here)
    const bool binned = fill_binned(p);
    BinArgs bin{};
    uint32_t bin_tiles = 0;
    if (binned) {
        const int rcb = bin_setup(p, &bin, &bin_tiles,
                                  {&p->d_pos, &p->d_vertex, &p->d_strand, &p->d_edges});
        if (rcb)
            return rcb;
    }

    // tile queues of the four tile kernels (tp_config.tile_queue)
    unsigned int *qbase = p->cfg.tile_queue ? p->d_queue.as<unsigned int>() : nullptr;

    // ---- a0: sentinels; with rounds, the class census and partition
    const bool graphs = p->cfg.graphs && rounds == 1;
    auto enqueue_a0 = [&](hipStream_t q) -> int {
        HIPCHK(launch_zero(cnt, sizeof(Counters), q));
        HIPCHK(launch_sentinels(W, a, p->d_sent_raw.p, p->d_sent.p, p->d_sent_owner.as<uint32_t>(),
                                sent_slots, p->d_pf.as<uint32_t>(), p->pf_log2, q));
        return TP_OK;
    };
    HIPCHK(hipEventRecord(p->ev[0], s));
    HIPCHK(hipMemcpyAsync(p->d_sets.p, desc.data(), nsets * sizeof(SetDesc),
                          hipMemcpyHostToDevice, s));
    if (rounds > 1) {
        int rc0 = enqueue_a0(s);
        if (rc0)
            return rc0;
        HIPCHK(p->d_census.ensure((uint64_t)nsets * CLASS_Q * 8));
        HIPCHK(launch_census(W, a, p->d_census.as<unsigned long long>(), p->grid[K_FILL], s));
        p->census.assign((size_t)nsets * CLASS_Q, 0);
        HIPCHK(hipMemcpyAsync(p->census.data(), p->d_census.p, p->census.size() * 8,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        p->bounds.assign((size_t)nsets * (rounds + 1), 0);
        for (uint32_t i = 0; i < nsets; ++i)
            class_partition(&p->census[(size_t)i * CLASS_Q], rounds,
                            &p->bounds[(size_t)i * (rounds + 1)]);
    }
    float ms_sent = 0, ms_fill = 0, ms_query = 0, ms_record = 0, ms_decide = 0, ms_pass2 = 0;

    uint64_t slots = 0;
    uint32_t attempts = 0;
    double est = 0;
    std::vector<uint32_t> hll(HLL_M);
    for (uint32_t round = 0; round < rounds; ++round) {
        // ---- a1-a2: first pass (of this round's class)
        if (rounds > 1) {
            for (uint32_t i = 0; i < nsets; ++i) {
                desc[i].cls_lo = p->bounds[(size_t)i * (rounds + 1) + round];
                desc[i].cls_hi = p->bounds[(size_t)i * (rounds + 1) + round + 1];
            }
            HIPCHK(hipMemcpyAsync(p->d_sets.p, desc.data(), nsets * sizeof(SetDesc),
                                  hipMemcpyHostToDevice, s));
        }
        // prologue (graph-replayable): sentinels on a single round, zeroing
        auto enqueue_p1 = [&](hipStream_t q) -> int {
            if (rounds == 1) {
                const int rc0 = enqueue_a0(q);
                if (rc0)
                    return rc0;
            }
            HIPCHK(launch_zero(scnt, nsets * sizeof(SetCounters), q));
            HIPCHK(launch_zero(p->d_hll.p, HLL_M * 4, q));
            if (!binned)  // the binned fill's first chunk writes every block
                HIPCHK(launch_zero(p->d_bloom.p, p->bloom_words * 4, q));
            if (qbase)  // the fill's and the query's tile queues
                HIPCHK(launch_zero(qbase, 2 * NXCD * sizeof(unsigned int), q));
            return TP_OK;
        };
        {
            KeyBuilder kb;
            kb(W)(a)(sa)(cnt)(scnt)(p->d_hll.p)(p->d_bloom.p)(p->bloom_words)(nsets)(
                p->d_sent_raw.p)(p->pf_log2)(p->d_sent_owner.p)(sent_slots)(binned)(qbase);
            const int rc1 = run_segment(p, graphs, 0, kb.v, s, enqueue_p1);
            if (rc1)
                return rc1;
        }
        // timed kernels, launched directly between their events
        HIPCHK(hipEventRecord(p->ev[1], s));
        if (binned)
            HIPCHK(launch_fill_binned(W, a, pool, cnt, bin, bin_tiles, s));
        else
            HIPCHK(launch_fill(W, with_queue(a, qbase, K_FILL, p->grid[K_FILL]), pool, cnt,
                               p->grid[K_FILL], s));
        HIPCHK(hipEventRecord(p->ev[2], s));
        HIPCHK(launch_query(W, with_queue(a, qbase, K_QUERY, p->grid[K_QUERY]), pool, sa,
                            p->d_c1.as<uint64_t>(),
                            c1u, round, cnt, p->d_hll.as<uint32_t>(), p->grid[K_QUERY], s));
        HIPCHK(launch_popcount(pool.words, p->bloom_words, p->d_bloom_starts.as<uint64_t>(),
                               nsets, scnt, s));
        HIPCHK(hipEventRecord(p->ev[3], s));
        HIPCHK(hipMemcpyAsync(hs.data(), scnt, nsets * sizeof(SetCounters),
                              hipMemcpyDeviceToHost, s));
        if (a.sketch)
            HIPCHK(hipMemcpyAsync(hll.data(), p->d_hll.p, HLL_M * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        float t1 = 0, t2 = 0;
        if (round == 0)
            HIPCHK(hipEventElapsedTime(&ms_sent, p->ev[0], p->ev[1]));
        HIPCHK(hipEventElapsedTime(&t1, p->ev[1], p->ev[2]));
        HIPCHK(hipEventElapsedTime(&t2, p->ev[2], p->ev[3]));
        ms_fill += t1;
        ms_query += t2;
        for (uint32_t i = 0; i < nsets; ++i) {
            tot[i].candidates += hs[i].candidates;
            tot[i].bloom_popcount += hs[i].bloom_popcount;
        }

        HIPCHK(hipEventRecord(p->ev[4], s));
        if (pass1_only) {
            for (uint32_t i = 0; i < nsets; ++i)
                tot[i].junctions += hs[i].candidates;
            for (int e = 5; e < 8; ++e)
                HIPCHK(hipEventRecord(p->ev[e], s));
            continue;
        }
        // ---- a3-a4: second pass over this round's candidates
        HIPCHK(p->d_j.ensure(p->bitmap_words * 8));
        if (a.sketch)
            est = hll_estimate(hll.data());
        const bool packed = table_packed(p);
        // wide keys with room in the top word carry their mask there
        const bool himask = table_himask(p);
        {
            // keys <= candidate positions; one set: the sketch's estimate
            // (+15% for its error) when smaller.  A table that overflows is
            // doubled and the pass repeated.
            std::vector<double> keys(nsets);
            for (uint32_t i = 0; i < nsets; ++i) {
                const double c = (double)std::max<uint64_t>(hs[i].candidates, 1);
                keys[i] = a.sketch ? std::min(c, est * 1.15) : c;
            }
            bool pow2 = true;
            const std::vector<uint64_t> caps = table_caps(p, keys, &pow2);
            p->table_pow2 = pow2;
            for (uint32_t i = 0; i < nsets; ++i)
                p->sets[i].table_cap = caps[i];
            // a table beyond the budget: Algorithm 3 with enough classes that
            // each round's table (about 1/rounds of this one) fits
            const uint64_t budget = p->cfg.table_budget;
            if (split && rounds == 1 && budget) {
                const uint64_t slot_bytes = 8ull * W + (packed || himask ? 0 : 1);
                uint64_t bytes = 0;
                for (uint32_t i = 0; i < nsets; ++i)
                    bytes += (caps[i] + TABLE_TAIL) * slot_bytes;
                if (bytes > budget) {
                    const double want = std::ceil(1.15 * (double)bytes / (double)budget);
                    *split = (uint32_t)std::min<double>(MAX_ROUNDS, std::max(2.0, want));
                    return RUN_SPLIT;
                }
            }
        }
        uint32_t round_attempts = 0;
        bool rbin_off = false;  // the binned record's scratch proved too small: direct
        for (;;) {
            ++attempts;
            ++round_attempts;
            slots = 0;
            for (auto &si : p->sets) {
                si.table_off = slots;
                slots += si.table_cap + TABLE_TAIL;
            }
            std::vector<SetDesc> d2 = set_descs(p);
            for (uint32_t i = 0; i < nsets; ++i) {
                d2[i].cls_lo = desc[i].cls_lo;
                d2[i].cls_hi = desc[i].cls_hi;
            }
            TableArgs t;
            t.packed = packed ? 1u : 0u;
            t.himask = himask ? 1u : 0u;
            // the last run's outputs are dead from here on: spare them if the
            // table does not fit beside them
            const std::initializer_list<DevBuf *> outputs = {&p->d_pos, &p->d_vertex, &p->d_strand,
                                                             &p->d_edges, &p->d_rbin};
            {
                const int rcr = reserve(p, {{&p->d_keys, slots * 8},
                                            {&p->d_masks, !packed && !himask ? slots : 0},
                                            {&p->d_keys_hi, W >= 2 ? slots * 8 : 0},
                                            {&p->d_keys_mid, W == 4 ? slots * 16 : 0}});
                if (rcr)
                    return rcr;
            }
            HIPCHK(ensure_spare(p->d_keys, slots * 8, outputs));
            if (!packed && !himask)
                HIPCHK(ensure_spare(p->d_masks, slots, outputs));
            if (W >= 2)
                HIPCHK(ensure_spare(p->d_keys_hi, slots * 8, outputs));
            if (W == 4)
                HIPCHK(ensure_spare(p->d_keys_mid, slots * 16, outputs));
            t.keys = p->d_keys.as<unsigned long long>();
            t.keys_hi = W >= 2 ? p->d_keys_hi.as<unsigned long long>() : nullptr;
            t.keys_mid = W == 4 ? p->d_keys_mid.as<unsigned long long>() : nullptr;
            t.masks = packed || himask ? nullptr : p->d_masks.as<uint32_t>();
            t.cap_m = t.cap_e = 0;  // per set, from its descriptor
            t.lomask = 0;
            t.pow2 = p->table_pow2 ? 1u : 0u;
            t.pad = 0;
            HIPCHK(hipMemcpyAsync(p->d_sets.p, d2.data(), nsets * sizeof(SetDesc),
                                  hipMemcpyHostToDevice, s));
            // binned record: one set, packed slots, home blocks of at most
            // 2^TABLE_BLOCK_LOG2 slots (the binned kernels take set 0's shape)
            RecBinArgs rb{};
            uint32_t rb_passes = 0;
            bool rbin = false;
            TableArgs t0 = t;
            if (!rbin_off && nsets == 1 && packed && d2[0].table_e <= TABLE_BLOCK_LOG2) {
                t0.cap_m = d2[0].table_m;
                t0.cap_e = d2[0].table_e;
                t0.lomask = (1ull << d2[0].table_e) - 1;
                const int rcb = rbin_setup(p, hs[0].candidates, d2[0].table_m,
                                           p->sets[0].table_cap * 8, &rb, &rb_passes, &rbin);
                if (rcb)
                    return rcb;
            }
            // prologue (graph-replayable): counters and the table cleared (the
            // binned record writes every block itself: only the spare tail)
            auto enqueue_p2 = [&](hipStream_t q) -> int {
                HIPCHK(launch_zero(&cnt->fill_atomics + PASS2_OFFSET,
                                   PASS2_FIELDS * sizeof(unsigned long long), q));
                HIPCHK(launch_zero(scnt, nsets * sizeof(SetCounters), q));
                if (rbin) {
                    TableArgs tail = t;
                    tail.keys = t.keys + p->sets[0].table_cap;
                    HIPCHK(launch_table_clear(W, tail, TABLE_TAIL, q));
                } else {
                    HIPCHK(launch_table_clear(W, t, slots, q));
                }
                if (qbase)  // the record's and the decision's tile queues
                    HIPCHK(launch_zero(qbase + 2 * NXCD, 2 * NXCD * sizeof(unsigned int), q));
                return TP_OK;
            };
            {
                KeyBuilder kb;
                kb(W)(t)(slots)(cnt)(scnt)(nsets)(qbase)(rbin);
                const int rc2 = run_segment(p, graphs, 1, kb.v, s, enqueue_p2);
                if (rc2)
                    return rc2;
            }
            HIPCHK(hipEventRecord(p->ev[5], s));
            if (rbin)
                HIPCHK(launch_record_binned(a, p->d_c1.as<uint64_t>(), t0, rb, rb_passes,
                                            d2[0].table_m, scnt, cnt, s));
            else
                HIPCHK(launch_record(W, with_queue(a, qbase, K_RECORD, p->grid[K_RECORD]),
                                     p->d_c1.as<uint64_t>(), t, cnt, p->grid[K_RECORD], s));
            HIPCHK(hipEventRecord(p->ev[6], s));
            HIPCHK(launch_decide(W, with_queue(a, qbase, K_DECIDE, p->grid[K_DECIDE]), sa,
                                 p->d_c1.as<uint64_t>(), t, p->d_j.as<uint64_t>(),
                                 round > 0, cnt, p->grid[K_DECIDE], s));
            HIPCHK(hipEventRecord(p->ev[7], s));
            std::vector<SetCounters> h2(nsets);
            unsigned long long rb_short = 0;
            HIPCHK(hipMemcpyAsync(&hc, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(h2.data(), scnt, nsets * sizeof(SetCounters),
                                  hipMemcpyDeviceToHost, s));
            if (rbin)
                HIPCHK(hipMemcpyAsync(&rb_short, rb.ctl + 1, sizeof(rb_short),
                                      hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            p->last_record_passes = rbin ? rb_passes : 0;
            if (rb_short) {
                // a pass had more items than the scratch holds (the table is
                // not complete): the same attempt again, recorded directly
                rbin_off = true;
                if (round_attempts >= MAX_ATTEMPTS)
                    return fail(TP_EOVERFLOW, "exact table overflowed after " +
                                                  std::to_string(round_attempts) + " attempts");
                continue;
            }
            bool overflow = false;
            for (uint32_t i = 0; i < nsets; ++i) {
                hs[i].junctions = h2[i].junctions;
                hs[i].table_keys = h2[i].table_keys;
                if (h2[i].overflow) {
                    overflow = true;
                    if (p->sets[i].table_cap >= MAX_TABLE)
                        return fail(TP_EOVERFLOW, "exact table of set " + std::to_string(i) +
                                                      " reached its size limit");
                    p->sets[i].table_cap = std::min(MAX_TABLE, 2 * p->sets[i].table_cap);
                }
            }
            if (!overflow) {
                p->last_cap.resize(nsets);
                p->last_off.resize(nsets);
                for (uint32_t i = 0; i < nsets; ++i) {
                    p->last_cap[i] = p->sets[i].table_cap;
                    p->last_off[i] = p->sets[i].table_off;
                }
                break;
            }
            if (round_attempts >= MAX_ATTEMPTS)
                return fail(TP_EOVERFLOW, "exact table overflowed after " +
                                              std::to_string(round_attempts) + " attempts");
        }
        if (hc.missing)
            return fail(TP_EDEVICE, "internal error: " + std::to_string(hc.missing) +
                                        " candidate k-mers missing from the exact table");
        float t3 = 0, t4 = 0, t5 = 0;
        HIPCHK(hipEventElapsedTime(&t3, p->ev[5], p->ev[6]));
        HIPCHK(hipEventElapsedTime(&t4, p->ev[6], p->ev[7]));
        HIPCHK(hipEventElapsedTime(&t5, p->ev[4], p->ev[7]));
        ms_record += t3;
        ms_decide += t4;
        ms_pass2 += t5;
        total_cnt.table_probes += hc.table_probes;
        for (uint32_t i = 0; i < nsets; ++i) {
            tot[i].junctions += hs[i].junctions;
            tot[i].table_keys += hs[i].table_keys;
            max_cap[i] = std::max(max_cap[i], p->sets[i].table_cap);
        }
    }
    p->jbits = pass1_only ? p->c1_out : p->d_j.as<uint64_t>();
    hs = tot;
    for (uint32_t i = 0; i < nsets; ++i)
        p->sets[i].table_cap = max_cap[i];
    HIPCHK(hipMemcpyAsync(&hc, cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    hc.table_probes = total_cnt.table_probes;

    // ---- a5: ordered compaction and edges
    uint64_t nj = 0;
    for (auto &c : hs)
        nj += c.junctions;
    if (nj < ns)
        return fail(TP_EDEVICE, "internal error: fewer junctions than strings");
    const uint64_t ne = nj - ns;
    const uint64_t nblocks = (p->bitmap_words + SCAN_WORDS - 1) / SCAN_WORDS;
    // the exact tables are dead from here on: spare them if the outputs do
    // not fit beside them (the next run allocates them again)
    const std::initializer_list<DevBuf *> tables = {&p->d_keys, &p->d_keys_hi, &p->d_keys_mid,
                                                    &p->d_masks};
    // the binned record's own scratch goes first when the outputs must grow
    if (p->d_rbin.p && (p->d_pos.cap < nj * 8 || p->d_vertex.cap < nj * 8 * W ||
                        p->d_strand.cap < nj || p->d_edges.cap < ne * sizeof(tp_edge)))
        p->d_rbin.release();
    {
        const int rcr = reserve(p, {{&p->d_pos, nj * 8}, {&p->d_vertex, nj * 8 * W},
                                    {&p->d_strand, nj}, {&p->d_edges, ne * sizeof(tp_edge)},
                                    {&p->d_joff, (ngen + 1) * 8}, {&p->d_blockcnt, nblocks * 4},
                                    {&p->d_blockoff, (nblocks + 1) * 8}});
        if (rcr)
            return rcr;
    }
    HIPCHK(ensure_spare(p->d_pos, nj * 8, tables));
    HIPCHK(ensure_spare(p->d_vertex, nj * 8 * W, tables));
    HIPCHK(ensure_spare(p->d_strand, nj, tables));
    HIPCHK(ensure_spare(p->d_edges, ne * sizeof(tp_edge), tables));
    // the table is still there unless it had to be freed for the outputs
    p->table_live = !pass1_only && p->d_keys.p != nullptr;
    HIPCHK(p->d_joff.ensure((ngen + 1) * 8));
    HIPCHK(p->d_blockcnt.ensure(nblocks * 4));
    HIPCHK(p->d_blockoff.ensure((nblocks + 1) * 8));
    OutArgs o;
    o.pos = p->d_pos.as<uint64_t>();
    o.vertex = p->d_vertex.as<uint64_t>();
    o.strand = p->d_strand.as<uint8_t>();
    o.joff = p->d_joff.as<uint64_t>();
    o.edges = p->d_edges.p;
    o.gbase = p->d_gbase.as<uint64_t>();
    o.n_genomes = (uint32_t)ngen;
    o.pad = 0;
    auto enqueue_compact = [&](hipStream_t q) -> int {
        HIPCHK(launch_compact(W, a, p->jbits, p->bitmap_words, p->d_blockcnt.as<uint32_t>(),
                              p->d_blockoff.as<uint64_t>(), o, nj, q));
        return TP_OK;
    };
    {
        KeyBuilder kb;
        kb(W)(a)(o)(p->jbits)(p->bitmap_words)(p->d_blockcnt.p)(p->d_blockoff.p)(nj);
        const int rc3 = run_segment(p, graphs, 2, kb.v, s, enqueue_compact);
        if (rc3)
            return rc3;
    }
    HIPCHK(hipEventRecord(p->ev[8], s));
    p->joff.assign(ngen + 1, 0);
    HIPCHK(hipMemcpyAsync(p->joff.data(), o.joff, (ngen + 1) * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    tp_stats &st = p->stats;
    st = tp_stats{};
    st.positions = p->positions;
    for (auto &c : hs) {
        st.candidates += c.candidates;
        st.bloom_popcount += c.bloom_popcount;
        st.table_keys += c.table_keys;
    }
    st.junctions = nj;
    st.edges = ne;
    st.table_capacity = 0;  // largest table of each set over the rounds, spare tails included
    for (const auto &si : p->sets)
        st.table_capacity += si.table_cap ? si.table_cap + TABLE_TAIL : 0;
    st.distinct_estimate = (uint64_t)est;
    st.table_attempts = attempts;
    st.sentinels = (uint32_t)(2 * ns);
    st.edge_positions = p->positions >= ns ? p->positions - ns : 0;
    st.fill_atomics = hc.fill_atomics;
    st.query_probes = hc.query_probes;
    st.table_probes = hc.table_probes;
    st.ms_sentinels = ms_sent;
    st.ms_fill = ms_fill;
    st.ms_query = ms_query;
    st.ms_record = ms_record;
    st.ms_decide = ms_decide;
    st.rounds = rounds;
    st.fill_chunks = binned ? (uint32_t)((p->n_tiles + bin_tiles - 1) / bin_tiles) : 0;
    st.record_passes = pass1_only ? 0 : p->last_record_passes;
    st.ms_pass1 = ms_sent + ms_fill + ms_query;
    st.ms_pass2 = ms_pass2;
    HIPCHK(hipEventElapsedTime(&st.ms_compact, p->ev[7], p->ev[8]));
    HIPCHK(hipEventElapsedTime(&st.ms_total, p->ev[0], p->ev[8]));
    p->set_cnt = hs;
    p->n_j = nj;
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

extern "C" int tp_get_set_stats(const tp_plan *p, uint32_t set, tp_stats *out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    if (set >= p->sets.size())
        return fail(TP_EINVAL, "set out of range");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    const SetInfo &si = p->sets[set];
    const SetCounters &c = p->set_cnt[set];
    const uint64_t nstr = si.str_hi - si.str_lo;
    *out = p->stats;  // batch-wide probes, estimate and device times
    out->positions = si.positions;
    out->candidates = c.candidates;
    out->junctions = p->joff[si.genome_hi] - p->joff[si.genome_lo];
    out->edges = out->junctions - nstr;
    out->bloom_popcount = c.bloom_popcount;
    out->table_capacity = si.table_cap ? si.table_cap + TABLE_TAIL : 0;
    out->table_keys = c.table_keys;
    out->sentinels = (uint32_t)(2 * nstr);
    out->edge_positions = si.positions >= nstr ? si.positions - nstr : 0;
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
    out->candidates = p->c1_out;
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
    uint8_t *m = (uint8_t *)host_alloc(total);
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

// Copy genomes [g0, g1) of the last run into a new host result, genome
// indices rebased to g0.  Their junctions are contiguous, and so are their
// edges: each string of c junctions has c - 1 edges, so the edges before
// genome g0 number (junctions before it) - (strings before it).
static int download_range(const tp_plan *p, uint32_t g0, uint32_t g1, uint32_t s0,
                          uint32_t s1, hipStream_t s, tp_result **out) {
    const uint64_t j0 = p->joff[g0], nj = p->joff[g1] - j0;
    const uint64_t e0 = j0 - s0, ne = nj - (s1 - s0);
    const uint32_t ng = g1 - g0;
    tp_result *r = alloc_result(ng, nj, ne, p->W);
    if (!r)
        return fail(TP_ENOMEM, "host allocation failed");
    r->n_genomes = ng;
    r->kmer_words = (uint32_t)p->W;
    r->k = p->k;
    r->flags = p->flags;
    r->n_junctions = nj;
    r->n_edges = ne;
    r->stats = p->stats;
    uint64_t *joff = (uint64_t *)r->junction_offset;
    for (uint32_t g = 0; g <= ng; ++g)
        joff[g] = p->joff[g0 + g] - j0;
    auto cp = [&](const void *dst, const DevBuf &src, uint64_t off, uint64_t bytes) {
        if (!bytes)
            return hipSuccess;
        return hipMemcpyAsync((void *)dst, (const uint8_t *)src.p + off, bytes,
                              hipMemcpyDeviceToHost, s);
    };
    hipError_t e = cp(r->junction_pos, p->d_pos, j0 * 8, nj * 8);
    if (e == hipSuccess)
        e = cp(r->vertex, p->d_vertex, j0 * 8 * p->W, nj * 8 * p->W);
    if (e == hipSuccess)
        e = cp(r->strand, p->d_strand, j0, nj);
    if (e == hipSuccess)
        e = cp(r->edges, p->d_edges, e0 * sizeof(tp_edge), ne * sizeof(tp_edge));
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        host_free(r);
        return fail(TP_EDEVICE, std::string("download: ") + hipGetErrorString(e));
    }
    if (g0) {
        tp_edge *ed = (tp_edge *)r->edges;
        for (uint64_t i = 0; i < ne; ++i)
            ed[i].genome -= g0;
    }
    *out = r;
    return TP_OK;
}

extern "C" int tp_download(const tp_plan *p, void *stream, tp_result **out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    *out = nullptr;
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    return download_range(p, 0, (uint32_t)p->n_bases.size(), 0, (uint32_t)p->strings.size(),
                          (hipStream_t)stream, out);
}

extern "C" int tp_download_set(const tp_plan *p, uint32_t set, void *stream, tp_result **out) {
    if (!p || !out)
        return fail(TP_EINVAL, "NULL argument");
    *out = nullptr;
    if (set >= p->sets.size())
        return fail(TP_EINVAL, "set out of range");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    const SetInfo &si = p->sets[set];
    int rc = download_range(p, si.genome_lo, si.genome_hi, si.str_lo, si.str_hi,
                            (hipStream_t)stream, out);
    if (rc == TP_OK)
        rc = tp_get_set_stats(p, set, &(*out)->stats);
    return rc;
}

extern "C" void twopaco_result_free(tp_result *r) { host_free(r); }

extern "C" int tp_debug_set_bloom(const tp_plan *p, uint32_t set, uint32_t *host_words,
                                  uint64_t n_words) {
    if (!p || !host_words)
        return fail(TP_EINVAL, "NULL argument");
    if (set >= p->sets.size())
        return fail(TP_EINVAL, "set out of range");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    const SetInfo &si = p->sets[set];
    if (n_words != si.b / 32)
        return fail(TP_EINVAL, "n_words must be the set's bloom_bits/32");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_words, p->d_bloom.as<uint32_t>() + si.bloom_off, n_words * 4,
                     hipMemcpyDeviceToHost));
    return TP_OK;
}

extern "C" int tp_debug_bloom(const tp_plan *p, uint32_t *host_words, uint64_t n_words) {
    return tp_debug_set_bloom(p, 0, host_words, n_words);
}

extern "C" int tp_debug_candidates(const tp_plan *p, uint64_t *host_words, uint64_t n_words) {
    if (!p || !host_words)
        return fail(TP_EINVAL, "NULL argument");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    if (n_words != p->bitmap_words)
        return fail(TP_EINVAL, "n_words must be tp_plan_bitmap_words()");
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(host_words, p->c1_out, n_words * 8, hipMemcpyDeviceToHost));
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

extern "C" int tp_debug_table(const tp_plan *p, uint32_t set, uint64_t *keys, uint8_t *masks,
                              uint64_t cap, uint64_t *n_out) {
    if (!p || !n_out)
        return fail(TP_EINVAL, "NULL argument");
    *n_out = 0;
    if (set >= p->sets.size())
        return fail(TP_EINVAL, "set out of range");
    if (!p->have_run)
        return fail(TP_ESTATE, "no completed run");
    if (!p->table_live || set >= p->last_cap.size())
        return fail(TP_ESTATE, "the last run kept no exact table (pass-1-only mode, or the "
                               "table was released to fit the outputs)");
    const uint64_t off = p->last_off[set], slots = p->last_cap[set] + TABLE_TAIL;
    const int W = p->W;
    const bool packed = table_packed(p), himask = table_himask(p);
    std::vector<uint64_t> lo(slots), hi, mid;
    std::vector<uint8_t> mk;
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(lo.data(), p->d_keys.as<uint64_t>() + off, slots * 8, hipMemcpyDeviceToHost));
    if (W >= 2) {
        hi.resize(slots);
        HIPCHK(hipMemcpy(hi.data(), p->d_keys_hi.as<uint64_t>() + off, slots * 8,
                         hipMemcpyDeviceToHost));
    }
    if (W == 4) {
        mid.resize(2 * slots);
        HIPCHK(hipMemcpy(mid.data(), p->d_keys_mid.as<uint64_t>() + 2 * off, slots * 16,
                         hipMemcpyDeviceToHost));
    }
    if (!packed && !himask) {
        mk.resize(slots);
        HIPCHK(hipMemcpy(mk.data(), p->d_masks.as<uint8_t>() + off, slots, hipMemcpyDeviceToHost));
    }
    // occupied slots: the key word (one word) or the top word (wide) is not empty
    uint64_t n = 0;
    for (uint64_t i = 0; i < slots; ++i)
        n += (W == 1 ? lo[i] : hi[i]) != EMPTY_KEY;
    *n_out = n;
    if (n > cap)
        return fail(TP_EINVAL, "cap is smaller than the number of table entries");
    if (n && (!keys || !masks))
        return fail(TP_EINVAL, "keys or masks is NULL");
    uint64_t e = 0;
    for (uint64_t i = 0; i < slots; ++i) {
        const uint64_t top = W == 1 ? lo[i] : hi[i];
        if (top == EMPTY_KEY)
            continue;
        uint64_t *kw = keys + e * W;
        uint8_t m = 0;
        if (W == 1) {
            kw[0] = packed ? top >> 8 : top;
            m = packed ? (uint8_t)(top & 0xFF) : mk[i];
        } else {
            kw[0] = lo[i];
            if (W == 4) {
                kw[1] = mid[2 * i];
                kw[2] = mid[2 * i + 1];
            }
            kw[W - 1] = himask ? top & HIKEY_BITS : top;
            m = himask ? (uint8_t)((top >> HIMASK_SHIFT) & 0xFF) : mk[i];
        }
        masks[e++] = m;
    }
    return TP_OK;
}

extern "C" int tp_build_batch(const tp_set *sets, uint32_t n_sets, uint32_t k,
                              uint32_t hash_count, uint32_t flags, tp_result **results) {
    if (!results)
        return fail(TP_EINVAL, "results is NULL");
    for (uint32_t i = 0; i < n_sets; ++i)
        results[i] = nullptr;
    tp_plan *p = nullptr;
    int rc = tp_batch_create(sets, n_sets, k, hash_count, flags, &p);
    if (rc)
        return rc;
    uint8_t *d_input = nullptr;
    hipError_t e = hipMalloc(&d_input, std::max<uint64_t>(p->input_bytes, 16));
    if (e != hipSuccess) {
        tp_plan_destroy(p);
        return fail(e == hipErrorOutOfMemory ? TP_ENOMEM : TP_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    rc = tp_batch_upload(p, sets, d_input, nullptr);
    if (!rc)
        rc = tp_run(p, d_input, nullptr);
    for (uint32_t i = 0; i < n_sets && !rc; ++i)
        rc = tp_download_set(p, i, nullptr, &results[i]);
    if (rc) {
        const std::string err = g_err;
        for (uint32_t i = 0; i < n_sets; ++i) {
            twopaco_result_free(results[i]);
            results[i] = nullptr;
        }
        g_err = err;
    }
    (void)hipFree(d_input);
    tp_plan_destroy(p);
    return rc;
}
