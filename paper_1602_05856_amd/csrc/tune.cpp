// Autotuner: picks a plan's runtime knobs (tp_config) by timing its kernels
// on its own input, and keeps the choice in a small text cache keyed by the
// device and the shape of the work.  Knobs change speed only, never results.
//
// A plan with auto-sized filters first gets its filter density (bits per
// (k+1)-mer, on the whole run: a denser filter costs pass 1 more cache
// misses, a sparser one lets more false candidates into pass 2).  With the
// blocked filter the atomic or binned fill is chosen next, on fill time,
// then the fill's deduplication (it
// changes the fill's LDS use, hence its occupancy), on fill time.  Each
// kernel is timed by its own HIP events (tp_stats), so one run under a
// given workgroups-per-CU value times all four tile kernels at that value,
// and each kernel keeps its own best.  Then the chunk size of the tile
// walks (tiles per workgroup visit) and the tile queue on the four kernels'
// time, then the first-pass tile order is
// chosen on fill + query time, the second-pass tile orders on record +
// decision time, the table load factor on the whole second
// pass (including any regrow-and-retry it causes), and graph replay on the
// whole run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "runtime.hpp"

using namespace tp;

namespace {

constexpr const char *CACHE_HEADER = "# twopaco autotune cache v1";

// Best of `reps` runs (the first run after a change may grow buffers).
int timed_run(tp_plan *p, const uint8_t *d_input, void *stream, int reps, tp_stats *best) {
    for (int r = 0; r < reps; ++r) {
        int rc = tp_run(p, d_input, stream);
        if (rc)
            return rc;
        tp_stats st;
        if ((rc = tp_get_stats(p, &st)))
            return rc;
        if (r == 0 || st.ms_total < best->ms_total)
            *best = st;
    }
    return TP_OK;
}

int cache_key(const tp_plan *p, std::string *key) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    char buf[256];
    bool any_auto = false;
    for (const auto &si : p->sets)
        any_auto |= si.b_auto;
    std::snprintf(buf, sizeof buf, "%s/cu%d/W%d/f%u/p%u/s%u%s", arch.c_str(),
                  prop.multiProcessorCount, p->W, p->flags, log2_ceil(p->positions + 1),
                  log2_ceil((uint64_t)p->sets.size()), any_auto ? "/auto" : "");
    *key = buf;
    return TP_OK;
}

bool parse_entry(const std::string &line, std::string *key, tp_config *c) {
    std::istringstream in(line);
    if (!(in >> *key >> c->wg_per_cu[0] >> c->wg_per_cu[1] >> c->wg_per_cu[2] >>
          c->wg_per_cu[3] >> c->tile_order >> c->table_load))
        return false;
    uint32_t graphs = 0, slabs = 0, dedup = 0, chunk = 0, bpe = 0, binned = 0, queue = 0;
    if (in >> graphs)  // optional fields
        c->graphs = graphs ? 1u : 0u;
    if (in >> slabs)
        c->pass2_slabs = slabs & 7u;
    if (in >> dedup)
        c->fill_dedup = dedup ? 1u : 0u;
    if (in >> chunk && chunk >= 1 && chunk <= 64)
        c->chunk_tiles = chunk;
    if (in >> bpe && bpe <= 256)
        c->bloom_bits_per_edge = bpe;
    if (in >> binned && binned <= 2)
        c->fill_binned = binned;
    if (in >> queue)
        c->tile_queue = queue ? 1u : 0u;
    return true;
}

std::string format_entry(const std::string &key, const tp_config &c) {
    char buf[384];
    std::snprintf(buf, sizeof buf, "%s %u %u %u %u %u %.3f %u %u %u %u %u %u %u", key.c_str(),
                  c.wg_per_cu[0], c.wg_per_cu[1], c.wg_per_cu[2], c.wg_per_cu[3], c.tile_order,
                  (double)c.table_load, c.graphs, c.pass2_slabs, c.fill_dedup, c.chunk_tiles,
                  c.bloom_bits_per_edge, c.fill_binned, c.tile_queue);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, tp_config *c) {
    std::ifstream in(path);
    std::string line, k;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#')
            continue;
        tp_config e = *c;  // fields the cache does not hold keep their values
        if (parse_entry(line, &k, &e) && k == key) {
            *c = e;
            return true;
        }
    }
    return false;
}

int cache_store(const char *path, const std::string &key, const tp_config &c) {
    std::vector<std::string> lines;
    {
        std::ifstream in(path);
        std::string line, k;
        while (std::getline(in, line)) {
            tp_config e = c;
            if (line.empty() || line[0] == '#' || !parse_entry(line, &k, &e) || k == key)
                continue;
            lines.push_back(line);
        }
    }
    lines.push_back(format_entry(key, c));
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out)
            return fail(TP_EINVAL, std::string("cannot write ") + tmp);
        out << CACHE_HEADER << "\n";
        for (const auto &l : lines)
            out << l << "\n";
        if (!out)
            return fail(TP_EINVAL, std::string("cannot write ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0)
        return fail(TP_EINVAL, std::string("cannot replace ") + path);
    return TP_OK;
}

}  // namespace

extern "C" int tp_autotune(tp_plan *p, const uint8_t *d_input, void *stream,
                           const char *cache_path, tp_config *out) {
    if (!p)
        return fail(TP_EINVAL, "plan is NULL");
    std::string key;
    int rc = cache_key(p, &key);
    if (rc)
        return rc;
    tp_config best = p->cfg;
    if (cache_path && cache_lookup(cache_path, key, &best)) {
        if ((rc = tp_plan_set_config(p, &best)))
            return rc;
        if (out)
            *out = p->cfg;
        return TP_OK;
    }
    const bool pass2 = (p->flags & TP_FLAG_PASS1_ONLY) == 0;

    // 0a. filter density of auto-sized filters, on the whole run; the
    //     default (16 bits per (k+1)-mer) unless another is 2% faster
    bool any_auto = false;
    for (const auto &si : p->sets)
        any_auto |= si.b_auto;
    if (any_auto) {
        const uint32_t dens[] = {16, 8, 32};
        float best_run = 1e30f;
        uint32_t best_bpe = 16;
        for (uint32_t d : dens) {
            tp_config c = best;
            c.bloom_bits_per_edge = d;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            if (st.ms_total < best_run * 0.98f) {
                best_run = st.ms_total;
                best_bpe = d;
            }
        }
        best.bloom_bits_per_edge = best_bpe;
    }

    // 0b. atomic or binned fill (blocked filter, binnable pool), on fill time
    if (fill_binnable(p)) {
        float ms[3] = {0, 0, 0};
        for (uint32_t v = 1; v <= 2; ++v) {
            tp_config c = best;
            c.fill_binned = v;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            ms[v] = st.ms_fill;
        }
        best.fill_binned = ms[2] < ms[1] * 0.98f ? 2u : 1u;
    }

    // 0c. fill deduplication (blocked filter, atomic fill), at the current
    //     workgroup counts
    if (p->flags & TP_FLAG_BLOCKED_FILTER) {
        float ms[2];
        for (uint32_t v = 0; v <= 1; ++v) {
            tp_config c = best;
            c.fill_dedup = v;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            ms[v] = st.ms_fill;
        }
        best.fill_dedup = ms[1] <= ms[0] ? 1u : 0u;
    } else {
        best.fill_dedup = 0;
    }

    // 1. workgroups per CU, per kernel
    const uint32_t occs[] = {0, 6, 4, 2};
    float best_ms[K_COUNT];
    for (auto &m : best_ms)
        m = 1e30f;
    for (uint32_t occ : occs) {
        tp_config c = best;
        for (auto &w : c.wg_per_cu)
            w = occ;
        if ((rc = tp_plan_set_config(p, &c)))
            return rc;
        tp_stats st;
        if ((rc = timed_run(p, d_input, stream, 2, &st)))
            return rc;
        const float ms[K_COUNT] = {st.ms_fill, st.ms_query, st.ms_record, st.ms_decide};
        for (int kid = 0; kid < K_COUNT; ++kid)
            if (ms[kid] < best_ms[kid] * 0.98f) {  // keep the larger grid unless 2% faster
                best_ms[kid] = ms[kid];
                best.wg_per_cu[kid] = occ;
            }
    }

    // 1b. chunk size of the tile walks (tiles per workgroup visit), on the
    //     four tile kernels together; the smallest chunk unless a larger one
    //     is 2% faster
    {
        const uint32_t chunks[] = {1, 2, 4, 8, 16};
        float best_ck = 1e30f;
        uint32_t best_chunk = best.chunk_tiles;
        for (uint32_t ck : chunks) {
            tp_config c = best;
            c.chunk_tiles = ck;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            const float ms = st.ms_fill + st.ms_query + st.ms_record + st.ms_decide;
            if (ms < best_ck * 0.98f) {
                best_ck = ms;
                best_chunk = ck;
            }
        }
        best.chunk_tiles = best_chunk;
    }

    // 1c. tile queue or static chunk schedule, on the four tile kernels
    //     together; the queue (the default) unless static is 2% faster
    {
        float ms[2] = {0, 0};
        for (uint32_t v = 0; v <= 1; ++v) {
            tp_config c = best;
            c.tile_queue = v;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            ms[v] = st.ms_fill + st.ms_query + st.ms_record + st.ms_decide;
        }
        best.tile_queue = ms[0] < ms[1] * 0.98f ? 0u : 1u;
    }

    // 2. first-pass tile order
    float best_p1 = 1e30f;
    uint32_t best_order = best.tile_order;
    for (uint32_t order = 0; order <= 1; ++order) {
        tp_config c = best;
        c.tile_order = order;
        if ((rc = tp_plan_set_config(p, &c)))
            return rc;
        tp_stats st;
        if ((rc = timed_run(p, d_input, stream, 2, &st)))
            return rc;
        if (st.ms_fill + st.ms_query < best_p1 * (order ? 0.98f : 1.0f)) {
            best_p1 = st.ms_fill + st.ms_query;
            best_order = order;
        }
    }
    best.tile_order = best_order;

    // 3. second-pass tile orders (record: memory order, first-pass order, or
    //    runs of it; decision: memory or first-pass order), on record +
    //    decision time together: the
    //    order the record leaves the table lines in the caches changes the
    //    decision's time, so the two bits are not chosen apart.  The default
    //    (decision only) is kept unless another is 2% faster.
    if (pass2) {
        const uint32_t orders[] = {2, 0, 3, 1, 6, 4};
        float best_ms2 = 1e30f;
        uint32_t best_slabs = best.pass2_slabs;
        for (uint32_t v : orders) {
            tp_config c = best;
            c.pass2_slabs = v;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            const float ms = st.ms_record + st.ms_decide;
            if (ms < best_ms2 * 0.98f) {
                best_ms2 = ms;
                best_slabs = v;
            }
        }
        best.pass2_slabs = best_slabs;
    }

    // 4. table load factor (whole second pass, regrowth included)
    if (pass2) {
        const std::vector<float> loads = p->sets.size() == 1
                                             ? std::vector<float>{0.25f, 0.35f, 0.5f, 0.7f, 0.9f}
                                             : std::vector<float>{0.5f, 1.0f, 2.0f, 4.0f};
        float best_p2 = 1e30f;
        float best_load = best.table_load;
        for (float load : loads) {
            tp_config c = best;
            c.table_load = load;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 2, &st)))
                return rc;
            if (st.ms_pass2 < best_p2 * 0.98f) {
                best_p2 = st.ms_pass2;
                best_load = load;
            }
        }
        best.table_load = best_load;
    }

    // 5. graph replay of the launch sequences (single round), on the whole run
    if (p->rounds == 1) {
        float ms[2] = {0, 0};
        for (uint32_t g = 0; g <= 1; ++g) {
            tp_config c = best;
            c.graphs = g;
            if ((rc = tp_plan_set_config(p, &c)))
                return rc;
            tp_stats st;
            if ((rc = timed_run(p, d_input, stream, 3, &st)))
                return rc;
            ms[g] = st.ms_total;
        }
        best.graphs = ms[1] < ms[0] * 0.99f ? 1u : 0u;
    }

    if ((rc = tp_plan_set_config(p, &best)))
        return rc;
    if ((rc = tp_run(p, d_input, stream)))
        return rc;
    if (cache_path && (rc = cache_store(cache_path, key, best)))
        return rc;
    if (out)
        *out = best;
    return TP_OK;
}
