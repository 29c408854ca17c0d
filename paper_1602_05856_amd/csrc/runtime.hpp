// Internal to the library: the plan object and the host helpers shared by
// the runtime (runtime.cpp) and the autotuner (tune.cpp).  Not part of the
// C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.hpp"
#include "twopaco.h"

namespace tp {

// Record `msg` as the calling thread's last error and return `code`.
int fail(int code, const std::string &msg);

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::tp::fail(e_ == hipErrorOutOfMemory ? TP_ENOMEM : TP_EDEVICE,          \
                              std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Device buffer that only grows (its contents do not survive a growth).
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

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline uint64_t pow2_ceil(uint64_t x) {
    uint64_t p = 1;
    while (p < x)
        p <<= 1;
    return p;
}

inline uint32_t log2_ceil(uint64_t x) {
    uint32_t l = 0;
    while ((1ull << l) < x)
        ++l;
    return l;
}

constexpr uint64_t MIN_TABLE = 1024;        // slots per set table
constexpr uint64_t MAX_TABLE = 1ull << 40;  // slots per set table
// Exact tables are rounded up to a power of two (the faster mode) unless that
// would leave more than this many bytes of slots unused across a run's sets.
constexpr uint64_t POW2_WASTE_BYTES = 4ull << 30;

// Capacity >= cap of the form m << e with m < 2^32 (the kernels take a home
// slot from m and e; see first_slot): one block of the next power of two
// (at least TABLE_ALIGN) up to 2^TABLE_BLOCK_LOG2 slots, else whole blocks of
// 2^TABLE_BLOCK_LOG2.  Idempotent, and doubling a shaped capacity keeps it
// shaped.
inline uint64_t shape_table(uint64_t cap, uint32_t *m, uint32_t *e) {
    const uint64_t blk = 1ull << TABLE_BLOCK_LOG2;
    if (cap <= blk) {
        uint32_t l = 0;
        while ((1ull << l) < std::max<uint64_t>(cap, TABLE_ALIGN))
            ++l;
        *m = 1;
        *e = l;
        return 1ull << l;
    }
    *m = (uint32_t)((cap + blk - 1) >> TABLE_BLOCK_LOG2);
    *e = TABLE_BLOCK_LOG2;
    return (uint64_t)*m << TABLE_BLOCK_LOG2;
}

constexpr uint32_t MAX_ATTEMPTS = 8;
constexpr uint32_t MAX_ROUNDS = 64;
constexpr uint64_t BLOOM_ALIGN_WORDS = 64;  // set filters start 256 bytes apart

// Host view of one set of a batch.
struct SetInfo {
    uint32_t genome_lo = 0, genome_hi = 0;  // its global genome indices
    uint32_t str_lo = 0, str_hi = 0;        // its strings
    uint64_t b = 0;                         // filter bits
    bool b_auto = false;                    // sized by the plan (bloom_bits_per_edge)
    uint64_t bloom_off = 0;                 // first 32-bit word in the filter pool
    uint64_t positions = 0;
    uint64_t table_cap = 0, table_off = 0;  // last run's table region
    uint64_t sent_tab_off = 0;              // its sentinel table: first slot, log2 size
    uint32_t sent_tab_log2 = 0;
};

// Sequence arguments of tile kernel kid with its tile queue (NXCD counters
// at qbase + kid * NXCD), or with the static schedule when qbase is null or
// the kernel has few tiles per workgroup of its grid.
SeqArgs with_queue(SeqArgs a, unsigned int *qbase, int kid, uint32_t grid);
// Whether the plan's fill can run binned (blocked filter, pool within the
// bucket limit).
bool fill_binnable(const tp_plan *p);
// Filter sizes of auto-sized sets (at p->cfg.bloom_bits_per_edge) and every
// set's offset in the filter pool.
void layout_filters(tp_plan *p);
// Default knobs: every resident workgroup slot, per-XCD slab order, and the
// table load factor of one set (sketch-sized) or of a batch (candidate-sized).
tp_config default_config(uint32_t n_sets);
// Rebuild the first-pass tile order for p->cfg.tile_order.
void build_tile_order(tp_plan *p);
// Lay out genome sets in an existing plan (as tp_batch_create does), keeping
// its device buffers, which only grow: a reused plan allocates no device
// memory once its buffers are large enough.  On failure the plan is empty.
void plan_clear_layout(tp_plan *p);
int plan_layout(tp_plan *p, const tp_set *sets, uint32_t n_sets, uint32_t k, uint32_t hash_count,
                uint32_t flags);
// Greedy class partition of per-subrange counters (CLASS_Q of them) into
// `classes` runs; bound gets classes + 1 subrange indices.
void class_partition(const uint64_t *e, uint32_t classes, uint32_t *bound);
// Exact-table capacities for per-set key counts at the plan's table_load:
// slots = keys / load, rounded up to a power of two unless that leaves more
// than POW2_WASTE_BYTES unused over all sets (then to the m << e shape);
// *pow2 receives the mode.  (tp_run sizes from candidate counts and the
// sketch, the caller-memory run from a stated bound.)
std::vector<uint64_t> table_caps(const tp_plan *p, const std::vector<double> &keys, bool *pow2);
// Table layout flags of a plan: packed one-word slots, mask in the top word.
bool table_packed(const tp_plan *p);
bool table_himask(const tp_plan *p);
// Set descriptors for given table capacities (offsets laid out in order).
std::vector<SetDesc> set_descs_for(const tp_plan *p, const std::vector<uint64_t> &caps, bool pow2,
                                   uint64_t *slots);
// Persistent grids of the tile kernels for the plan's knobs (needs the device).
int plan_grids(tp_plan *p, int dev);
// Caller-memory run: write the layout tables into a workspace, and enqueue a
// whole run on it (no host wait, no allocation).
int ws_prepare(tp_plan *p, uint8_t *base, hipStream_t s);
int ws_run(tp_plan *p, const uint8_t *d_input, uint8_t *base, uint8_t *outb, hipStream_t s);
// Device bytes the plan's buffers hold now.
uint64_t plan_device_bytes(const tp_plan *p);
// Free the plan's device buffers (they are allocated again on the next run).
void plan_release(tp_plan *p);

}  // namespace tp

namespace tp {
// A launch sequence captured as a HIP graph, keyed by the bytes of every
// argument it was captured with.
struct Segment {
    hipGraphExec_t exec = nullptr;
    std::vector<uint8_t> key;
};

// Layout of a caller-owned workspace and output buffer (tp_run_ws): byte
// offsets of every region, the table capacities from the stated bound, and
// the set descriptors written into the workspace.
struct WsState {
    bool valid = false;
    uint64_t gen = 0;                 // plan layout generation it was made for
    const void *prepared = nullptr;   // workspace last prepared for it
    tp_ws_layout pub{};               // the public part (sizes, offsets)
    uint64_t o_tiles = 0, o_tile_info = 0, o_sets = 0, o_bloom_starts = 0, o_strings = 0,
             o_gbase = 0, o_sent_raw = 0, o_sent = 0, o_sent_owner = 0, o_pf = 0, o_bloom = 0,
             o_c1 = 0, o_c1u = 0,
             o_j = 0, o_cnt = 0, o_set_cnt = 0, o_census = 0, o_bounds = 0, o_keys = 0,
             o_keys_hi = 0, o_keys_mid = 0, o_masks = 0, o_blockcnt = 0, o_blockoff = 0,
             o_queue = 0;
    uint64_t slots = 0, nblocks = 0;
    bool pow2 = true, packed = false, himask = false;
    std::vector<SetDesc> desc;
    std::vector<uint64_t> bloom_starts;
    uint32_t grid[K_COUNT] = {};
};
}  // namespace tp

// The plan behind the opaque tp_plan handle of the C ABI.
struct tp_plan {
    uint32_t k = 0, h = 0, flags = 0;
    int W = 1;
    std::vector<tp::SetInfo> sets;
    std::vector<uint64_t> n_bases, gbase;  // per global genome
    std::vector<tp::DString> strings;
    std::vector<uint32_t> tile_order;      // first-pass order: per XCD, set by set, slab by slab
    std::vector<tp::TileInfo> tile_info;       // per tile: set and string range
    std::vector<uint64_t> bloom_starts;    // per set: first filter word; then the pool size
    uint64_t xcd_start[tp::NXCD + 1] = {};
    uint64_t total = 0, n_tiles = 0, bitmap_words = 0, input_bytes = 0, positions = 0;
    uint64_t bloom_words = 0;              // filter pool, 32-bit words
    uint64_t sent_tab_slots = 0;           // sentinel-table pool, slots (even)
    uint32_t pf_log2 = 10;
    uint32_t grid[tp::K_COUNT] = {};           // persistent grid per tile kernel (0: not set)
    uint32_t n_cu = 0;                     // CUs the plan's kernels run on (set with the grids)
    uint32_t rounds = 1;                   // Algorithm 3: k-mer classes, one round each
    uint32_t last_rounds = 1;              // rounds of the last run (more with a table budget)
    // Called before a run grows its device buffers, with the bytes the plan
    // will hold after the growth (a server's budget check); a status other
    // than TP_OK fails the run.
    int (*grow_hook)(void *ctx, uint64_t bytes) = nullptr;
    void *grow_ctx = nullptr;
    uint32_t cu_limit = 0;                 // CUs its stream may use (0: all); sizes the grids
    tp_config cfg{};                       // runtime knobs (autotuner)

    int device = -1;
    bool static_uploaded = false;
    bool order_uploaded = false;           // tile_order on the device matches cfg
    tp::DevBuf d_tiles, d_tile_info, d_sets, d_bloom_starts, d_strings, d_gbase;
    tp::DevBuf d_sent_raw, d_sent, d_sent_owner, d_pf, d_bloom, d_c1, d_j, d_cnt, d_set_cnt, d_hll;
    tp::DevBuf d_keys, d_keys_hi, d_keys_mid, d_masks, d_blockcnt, d_blockoff;
    tp::DevBuf d_pos, d_vertex, d_strand, d_edges, d_joff;
    tp::DevBuf d_c1u, d_census;            // rounds: union of candidates, class census
    tp::DevBuf d_bin;                      // binned fill: counts, offsets, region starts
    tp::DevBuf d_queue;                    // tile queues of the four tile kernels
    tp::DevBuf d_rbin;                     // binned record: items (when the outputs cannot hold them)
    std::vector<uint64_t> census;          // rounds: per set, CLASS_Q counters
    std::vector<uint32_t> bounds;          // rounds: per set, rounds + 1 class bounds
    // run timeline: 0 start, 1 sentinels, 2 fill, 3 query, 4 pass 2 start,
    // 5 record start, 6 record end, 7 decide end, 8 compaction end
    hipEvent_t ev[9] = {};
    tp::Segment seg[3];                    // graphs: first pass, second pass, compaction
    hipStream_t cap = nullptr;             // graphs: capture stream

    bool have_run = false;
    bool table_pow2 = true;  // table mode of the last sizing (every set 2^e, else m << e)
    std::vector<uint64_t> last_cap, last_off;  // last table attempt: per-set capacity, offset
    bool table_live = false;  // the last run's table is still in d_keys..
    uint32_t last_record_passes = 0;  // binned record: passes of the last table attempt
    uint64_t layout_gen = 1;  // bumped by changes that invalidate a workspace layout
    tp::WsState ws;           // caller-memory run
    tp_stats stats{};
    std::vector<tp::SetCounters> set_cnt;  // last run, per set
    std::vector<uint64_t> joff;        // last run, per-genome junction offsets
    uint64_t n_j = 0, n_e = 0;
    uint64_t *jbits = nullptr;  // J bitmap of the last run (C1 in pass-1-only mode)
    uint64_t *c1_out = nullptr; // candidate bitmap of the last run (union over rounds)

    template <class F> void for_each_buf(F f) {
        for (tp::DevBuf *b : {&d_tiles, &d_tile_info, &d_sets, &d_bloom_starts, &d_strings,
                              &d_gbase, &d_sent_raw, &d_sent, &d_sent_owner, &d_pf, &d_bloom,
                              &d_c1, &d_j,
                              &d_cnt, &d_set_cnt, &d_hll, &d_keys, &d_keys_hi, &d_keys_mid, &d_masks,
                              &d_blockcnt, &d_blockoff, &d_pos, &d_vertex, &d_strand,
                              &d_edges, &d_joff, &d_c1u, &d_census, &d_bin, &d_queue, &d_rbin})
            f(*b);
    }

    void drop_graphs() {
        for (auto &g : seg) {
            if (g.exec)
                (void)hipGraphExecDestroy(g.exec);
            g.exec = nullptr;
            g.key.clear();
        }
    }

    ~tp_plan() {
        drop_graphs();
        if (cap)
            (void)hipStreamDestroy(cap);
        for (auto &e : ev)
            if (e)
                (void)hipEventDestroy(e);
    }
};

