// Data layout in HBM and the kernel launch interface shared by the host
// runtime and the gfx950 kernels.
//
// A plan holds one or more independent genome sets (a batch); a plain build
// is a batch of one set.  Global base index: all genomes of all sets live in
// one 2-bit packed buffer, genome g starting at base index gbase[g], a
// multiple of TILE (so every tile belongs to one genome, hence one set).
// Position bitmaps (candidates C1, junctions J) have one bit per global base
// index; bit i of 64-bit word w is index 64*w + i.  Work is cut into tiles of
// TILE consecutive indices; a tile's bitmap words are written by the wave
// that owns them, so no bitmap atomics are needed.  Each set has its own
// Bloom filter, sentinel list and exact table, carved out of shared pools and
// described by a SetDesc.
//
// Tile order of the first pass: homologous tiles (the same offset in every
// genome) form a slab; slab s goes to XCD s mod 8, and the workgroups of one
// XCD walk its slabs in order, so the filter lines probed by similar genomes
// at similar offsets are fetched into that XCD's L2 once and then hit there.
// The second pass walks tiles in memory order, in that order, or in runs of
// it (tp_config.pass2_slabs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tp {

constexpr uint32_t TILE = 2048;                    // positions per tile
constexpr uint32_t TILE_WORDS = TILE / 32;         // packed 64-bit words per tile
constexpr uint32_t STAGE_WORDS = TILE_WORDS + 6;   // + 1 word before, 5 after (128-base windows)
constexpr uint32_t BLOCK = 256;                    // threads per workgroup
constexpr uint32_t GENOME_ALIGN = TILE;            // bases
constexpr uint32_t NXCD = 8;                       // accelerator dies (L2 domains)
constexpr uint32_t HLL_LOG2 = 12;                  // distinct-count sketch registers
constexpr uint32_t HLL_M = 1u << HLL_LOG2;
constexpr uint32_t PF_MAX_LOG2 = 16;               // sentinel prefilter bits (max)
constexpr uint32_t SCAN_WORDS = 2048;              // bitmap words per compaction block
constexpr uint32_t FILL_CHUNK = 8;                 // deduplicating fill: tiles per visit
constexpr uint32_t RECORD_RUN = 8;                 // record in runs: tiles per visit
constexpr uint32_t FILL_DD = 4096;                 // deduplicating fill: LDS table entries
constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr uint64_t PENDING_BIT = 1ull << 63;       // two-word keys: high word claimed
constexpr uint32_t MAX_PROBE = 1u << 12;           // exact-table probe bound (then regrow)
constexpr uint64_t TABLE_ALIGN = 64;               // set tables start and end on 512-byte key rows
constexpr uint64_t TABLE_TAIL = MAX_PROBE;         // spare slots past a set's capacity (never probed)
constexpr uint32_t TABLE_BLOCK_LOG2 = 13;          // any-size tables: blocks of 8192 slots (probes wrap)
static_assert(TABLE_TAIL % TABLE_ALIGN == 0, "set regions stay aligned");
constexpr uint32_t CLASS_Q_LOG2 = 10;              // k-mer class subranges (rounds)
constexpr uint32_t CLASS_Q = 1u << CLASS_Q_LOG2;
// Binned fill (blocked filter): the filter pool in regions of BIN_REGION
// blocks (one workgroup's LDS), BIN_SUB regions to a bucket.
constexpr uint32_t BIN_REGION_LOG2 = 13;           // 8192 blocks = 64 KiB
constexpr uint32_t BIN_REGION = 1u << BIN_REGION_LOG2;
constexpr uint32_t BIN_SUB_LOG2 = 9;
constexpr uint32_t BIN_SUB = 1u << BIN_SUB_LOG2;
constexpr uint32_t BIN_MAX_BUCKETS = 1024;         // pools up to 2^32 blocks (32 GiB)
constexpr uint32_t BIN_SPLIT_BLOCK = 1024;         // threads of the bucket split
constexpr uint32_t BIN_SCAN_BLOCK = 1024;          // threads of the offset scan
constexpr uint32_t BIN_CHUNK_TILES_MAX = 1u << 20; // 2^31 positions per chunk (explicit)
constexpr uint32_t BIN_SPLIT_PER = 16;             // bucket split: items per thread per batch
constexpr uint32_t BIN_SCATTER_PER = 16;           // bucket scatter: items per thread per batch
constexpr uint32_t BIN_SCATTER_BLOCK = 1024;       // bucket scatter: threads per workgroup
constexpr uint32_t BIN_APPLY_BLOCK = 1024;         // threads of a region's (a block's) apply
constexpr uint32_t BIN_WG_PER_CU = 8;              // count and scatter workgroups per CU

// A string of S: a maximal N-free run of one genome, of length >= k.
struct DString {
    uint64_t gstart;  // global base index of its first base
    uint64_t gend;    // one past its last base
    uint32_t genome;  // global genome index (over all sets)
    uint32_t set;
};

// Per-tile facts computed on the host: its set and the strings that hold
// positions in it (so no tile kernel searches the string list).
struct TileInfo {
    uint32_t set;
    uint32_t str_lo, str_hi;  // strings overlapping [tile * TILE, (tile + 1) * TILE)
    uint32_t pad;
};

struct SetDesc {
    uint64_t bloom_off;         // first 32-bit word of its filter in the filter pool
    uint64_t bloom_mask;        // filter bits - 1
    uint64_t table_off;         // first slot of its table in the table pools (multiple of 64)
    uint64_t sent_tab_off;      // first slot of its sentinel table in the sentinel pool
    uint32_t table_m, table_e;  // its table has m << e home slots (region: + TABLE_TAIL)
    uint32_t sent_lo, sent_hi;  // its slice of the sentinel array (2 per string)
    uint32_t str_lo, str_hi;    // its strings
    uint32_t cls_lo, cls_hi;    // current round: class subranges [cls_lo, cls_hi)
    uint32_t sent_tab_log2;     // its sentinel table has 2^log2 slots (at most half full)
    uint32_t pad;
};

// Device counters of one run, per set.
struct SetCounters {
    unsigned long long candidates;  // |C1|
    unsigned long long bloom_popcount;
    // second-pass fields, cleared before every table attempt
    unsigned long long junctions;   // |J|
    unsigned long long table_keys;  // keys claimed in the exact table
    unsigned long long overflow;    // probe bound or spin bound hit
    unsigned long long pad[3];
};
constexpr uint32_t SET_PASS2_OFFSET = 2;  // first second-pass field
constexpr uint32_t SET_PASS2_FIELDS = 3;

// Device counters of one run, whole batch.
struct Counters {
    unsigned long long fill_atomics;  // filter atomicOr issued
    unsigned long long query_probes;  // filter words loaded by the query
    // second-pass fields, cleared before every table attempt
    unsigned long long table_probes;  // slots visited by record + decision
    unsigned long long missing;       // candidate k-mers not found (must stay 0)
    unsigned long long pad[4];
};
constexpr uint32_t PASS2_OFFSET = 2;
constexpr uint32_t PASS2_FIELDS = 2;

struct SeqArgs {
    const uint64_t *seq;       // packed input as 64-bit words
    uint64_t seq_words;
    const DString *strings;
    uint32_t n_strings;
    uint32_t k;
    uint64_t n_tiles;
    uint32_t single;           // ordinary graph only (no reverse complements)
    uint32_t sketch;           // keep the distinct-count sketch (batches of one set)
    const uint32_t *tile_order;    // first-pass order: tiles grouped per XCD, slab by slab
    uint64_t xcd_start[NXCD + 1];  // tile_order range of each XCD
    const TileInfo *tiles;         // per tile, in memory order
    const SetDesc *sets;
    SetCounters *set_cnt;
    uint32_t n_sets;
    uint32_t classes;          // multiple rounds: only k-mers of the round's class count
    uint32_t pass2_slabs;      // bit 0 record, bit 1 decision: walk the first-pass order;
                               // bit 2 record in runs of RECORD_RUN entries of it
    uint32_t fill_dedup;       // blocked fill: skip filter effects the workgroup has sent
    uint32_t chunk;            // tiles a workgroup takes per visit of a tile walk
    uint32_t pad;
    unsigned int *queue;       // tile queue of this launch (NXCD zeroed counters), or
                               // null: the walk's static chunk schedule
};

enum KernelId { K_FILL = 0, K_QUERY = 1, K_RECORD = 2, K_DECIDE = 3, K_COUNT = 4 };

// Sentinel k-mers: per set an open-addressing table of the normalised first
// and last k-mers of its strings (home slot by hash, linear probing, empty
// slots all ones -- never a k-mer value), plus one bit prefilter for all
// sets kept in LDS.
struct SentArgs {
    const void *table;         // sentinel-table pool: W words per slot
    uint32_t n;                // sentinel k-mers (2 per string)
    uint32_t pf_log2;          // prefilter size, log2 bits
    const uint32_t *prefilter;
};
constexpr uint32_t SENT_TAB_MIN_LOG2 = 4;

struct BloomArgs {
    uint32_t *words;           // bit i: bit (i & 31) of words[i >> 5] (pool, or a set's region)
    uint64_t mask;             // bits - 1 (bits a power of two)
    uint32_t h;                // hash functions
    uint32_t blocked;          // blocked layout: 64-bit blocks keyed by the middle (k-1)-mer
};

// Exact-table layouts:
//   packed (k <= 27): one 64-bit word per slot, key << 8 | in/out mask
//   split  (k <= 31): key words + 8-bit masks packed 4 per 32-bit word
//   wide   (k <= 63): low and high key words + masks
//   wide4  (k <= 127): low, middle (2 per slot) and top key words + masks
// Pointers are the pools' bases; a tile's set shifts them by table_off.
struct TableArgs {
    unsigned long long *keys;     // slot words (packed) / key or low key words
    unsigned long long *keys_hi;  // top key words (two and four words), else null
    unsigned long long *keys_mid; // four-word keys: words 1 and 2, two per slot, else null
    uint32_t *masks;              // split and wide layouts (not himask)
    uint64_t lomask;              // (1 << cap_e) - 1 (a set's; filled per tile)
    uint32_t cap_m, cap_e;        // a set's capacity: cap_m << cap_e home slots
    uint32_t packed;
    uint32_t himask;              // wide keys: the mask in bits HIMASK_SHIFT.. of keys_hi
    uint32_t pow2;                // table mode: every set's capacity is 2^cap_e (cap_m = 1)
    uint32_t pad;
};
constexpr uint32_t PACKED_MAX_K = 27;  // 2k + 8 <= 62 bits
// Wide keys whose top word has at most HIMASK_SHIFT key bits keep their edge
// mask in that word, above the key bits (the pending bit stays bit 63).
constexpr uint32_t HIMASK_SHIFT = 54;
constexpr uint64_t HIKEY_BITS = (1ull << HIMASK_SHIFT) - 1;

struct OutArgs {
    uint64_t *pos;             // genome coordinate per junction
    uint64_t *vertex;          // W words per junction
    uint8_t *strand;
    uint64_t *joff;            // n_genomes + 1
    void *edges;               // tp_edge per edge
    const uint64_t *gbase;     // per genome
    uint32_t n_genomes;
    uint32_t pad;
};

// -------------------------------------------------------------- launchers
// Resident workgroups per CU of a tile kernel (sizes its persistent grid):
// pass1_occupancy for K_FILL / K_QUERY, pass2_occupancy for K_RECORD / K_DECIDE.
hipError_t pass1_occupancy(KernelId which, int W, bool blocked, bool fill_dedup,
                           int *blocks_per_cu);
hipError_t pass2_occupancy(KernelId which, int W, int *blocks_per_cu);
hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

// a0: normalised first/last k-mer of every string (raw: 2 per string), each
// set's sentinel table (values, and a claim word per slot; tab_slots in all)
// and the sentinel prefilter.
hipError_t launch_sentinels(int W, const SeqArgs &a, void *raw, void *tab, uint32_t *tab_owner,
                            uint64_t tab_slots, uint32_t *prefilter, uint32_t pf_log2,
                            hipStream_t s);
// a1: insert every normalised (k+1)-mer into its set's Bloom filter.
// Binned fill of a blocked filter pool (the same bits as launch_fill): per
// chunk of tiles, every edge's filter effect becomes one 64-bit item
// (global block << 16 | offset | stride << 6 | pair << 12), the items are
// staged in position order, partitioned by bucket and then by region in two
// streaming passes, and one workgroup per region applies its items to the
// region with LDS atomics and writes it back.  Scratch: items_a and items_b
// hold one slot per position of a chunk; counts and offsets one entry per
// (bucket, workgroup), region_off one per region of the last bucket rounded
// up.
struct BinArgs {
    uint64_t *items_a;         // chunk items by bucket
    uint64_t *items_b;         // chunk items in position order, then by region (4-byte)
    uint32_t *counts;          // [bucket * grid + workgroup]
    uint64_t *offsets;         // exclusive scan of counts, n + 1 entries
    uint64_t *region_off;      // per region: first item in items_b; then the total
    uint64_t tile_lo, tile_hi; // the chunk's tiles, memory order
    uint64_t n_blocks;         // 64-bit blocks of the filter pool
    uint32_t n_buckets;        // ceil(regions / BIN_SUB)
    uint32_t grid;             // workgroups of the count and scatter kernels
    uint32_t first;            // first chunk: regions start from zero
    uint32_t pad;
};
hipError_t launch_fill_binned(int W, const SeqArgs &a, const BloomArgs &pool, Counters *cnt,
                              BinArgs b, uint32_t tiles_per_chunk, hipStream_t s);
hipError_t launch_fill(int W, const SeqArgs &a, const BloomArgs &pool, Counters *cnt,
                       uint32_t grid, hipStream_t s);
// a2: Bloom-queried neighbourhood of every k-mer position -> C1 bitmap,
// candidate counts and (one set) distinct-count sketch of candidate k-mers.
// With classes, only the round's k-mers are evaluated, and c1_union (when
// not null) collects the rounds' candidate bitmaps (overwritten in round 0).
hipError_t launch_query(int W, const SeqArgs &a, const BloomArgs &pool, const SentArgs &sa,
                        uint64_t *c1, uint64_t *c1_union, uint32_t round, Counters *cnt,
                        uint32_t *hll, uint32_t grid, hipStream_t s);
// Multiple rounds: per set, CLASS_Q counters of (k+1)-mer occurrences per
// class subrange of the two k-mers each contains (once per distinct one).
hipError_t launch_census(int W, const SeqArgs &a, unsigned long long *counters, uint32_t grid,
                         hipStream_t s);
// Filter popcount per set (bloom_starts: n_sets + 1 word offsets, device).
hipError_t launch_popcount(const uint32_t *pool, uint64_t n_words, const uint64_t *bloom_starts,
                           uint32_t n_sets, SetCounters *set_cnt, hipStream_t s);
// a3: exact in/out edge masks of every candidate k-mer.
hipError_t launch_table_clear(int W, const TableArgs &pool, uint64_t slots, hipStream_t s);
hipError_t launch_record(int W, const SeqArgs &a, const uint64_t *c1, const TableArgs &pool,
                         Counters *cnt, uint32_t grid, hipStream_t s);

// Binned record (one set, packed one-word slots, home blocks of at most
// 2^TABLE_BLOCK_LOG2 slots): per pass, the candidates whose home block lies
// in [r_lo, r_hi) become items (their slot words), are partitioned by block
// and each block is built in LDS and written out whole.
constexpr uint32_t RBIN_SEG = 16384;   // staging items a count workgroup claims at once
constexpr uint32_t RBIN_MAX_PASSES = 64;
struct RecBinArgs {
    uint64_t *items_a;         // the pass's items by bucket
    uint64_t *items_b;         // staging (segments), then the items by block
    uint32_t *counts;          // [bucket * grid + workgroup]
    uint64_t *offsets;         // exclusive scan of counts, n + 1 entries
    uint64_t *region_off;      // per block of the pass: first item in items_b; then the total
    unsigned long long *ctl;   // [0] staging items claimed, [1] nonzero: scratch too small
    uint64_t cap;              // items each of items_a and items_b hold
    uint64_t r_lo, r_hi;       // the pass's home blocks
    uint32_t n_buckets;        // ceil((r_hi - r_lo) / BIN_SUB)
    uint32_t grid;             // workgroups of the count, histogram and scatter kernels
};
// table: set 0's table (keys, cap_m, cap_e, lomask, pow2 filled in).
hipError_t launch_record_binned(const SeqArgs &a, const uint64_t *c1, const TableArgs &table,
                                RecBinArgs rb, uint32_t passes, uint64_t n_blocks,
                                SetCounters *set_cnt, Counters *cnt, hipStream_t s);
// a4: junction decision for every candidate -> J bitmap and counts.
// With accumulate, junction words are ORed into jbits (rounds after the first).
hipError_t launch_decide(int W, const SeqArgs &a, const SentArgs &sa, const uint64_t *c1,
                         const TableArgs &pool, uint64_t *jbits, bool accumulate, Counters *cnt,
                         uint32_t grid, hipStream_t s);
// a5: ordered compaction of J and compacted edges.
hipError_t launch_compact(int W, const SeqArgs &a, const uint64_t *jbits, uint64_t nwords,
                          uint32_t *blockcnt, uint64_t *blockoff, const OutArgs &o,
                          uint64_t n_junctions, hipStream_t s);
// a5 with the junction count unknown on the host: the kernels always run,
// writing at most max_j junctions and max_e edges (joff holds true counts).
hipError_t launch_compact_bound(int W, const SeqArgs &a, const uint64_t *jbits, uint64_t nwords,
                                uint32_t *blockcnt, uint64_t *blockoff, const OutArgs &o,
                                uint64_t max_j, uint64_t max_e, hipStream_t s);

// Multiple rounds on the device: the greedy partition of every set's census
// (bounds: rounds + 1 per set), and the round's class bounds copied into the
// set descriptors.
hipError_t launch_partition(const unsigned long long *census, uint32_t n_sets, uint32_t rounds,
                            uint32_t *bounds, hipStream_t s);
hipError_t launch_set_round(SetDesc *sets, const uint32_t *bounds, uint32_t n_sets,
                            uint32_t rounds, uint32_t round, hipStream_t s);

// Counts of a caller-memory run, summed on the device (tp_ws_counts layout:
// status, positions, candidates, junctions, edges, table_keys, popcount).
struct FinalizeArgs {
    const SetCounters *set_cnt;
    const Counters *cnt;
    const uint64_t *blockoff;  // compaction scan: total at [nblocks]
    uint64_t nblocks;
    uint32_t n_sets;
    uint32_t pass2;            // second pass ran (table status is meaningful)
    uint64_t n_strings, positions, max_j;
    unsigned long long *out;   // 16 words
};
hipError_t launch_ws_finalize(const FinalizeArgs &f, hipStream_t s);

}  // namespace tp
