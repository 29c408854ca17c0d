// Data layout in HBM and the kernel launch interface shared by the host
// runtime and the gfx950 kernels.
//
// Global base index: all genomes of a plan live in one 2-bit packed buffer,
// genome g starting at base index gbase[g], a multiple of TILE (so every tile
// belongs to one genome).  Position bitmaps (candidates C1, junctions J) have
// one bit per global base index; bit i of 64-bit word w is index 64*w + i.
// Work is cut into tiles of TILE consecutive indices; a tile's bitmap words
// are written by the wave that owns them, so no bitmap atomics are needed.
//
// Tile order of the first pass: homologous tiles (the same offset in every
// genome) form a slab; slab s goes to XCD s mod 8, and the workgroups of one
// XCD walk its slabs in order, so the filter lines probed by similar genomes
// at similar offsets are fetched into that XCD's L2 once and then hit there.
// The second pass walks tiles in plain order (see linear_cursor).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tp {

constexpr uint32_t TILE = 2048;                    // positions per tile
constexpr uint32_t TILE_WORDS = TILE / 32;         // packed 64-bit words per tile
constexpr uint32_t STAGE_WORDS = TILE_WORDS + 4;   // + 1 word before, 3 after
constexpr uint32_t BLOCK = 256;                    // threads per workgroup
constexpr uint32_t GENOME_ALIGN = TILE;            // bases
constexpr uint32_t NXCD = 8;                       // accelerator dies (L2 domains)
constexpr uint32_t HLL_LOG2 = 12;                  // distinct-count sketch registers
constexpr uint32_t HLL_M = 1u << HLL_LOG2;
constexpr uint32_t PF_MAX_LOG2 = 15;               // sentinel prefilter bits (max)
constexpr uint32_t SCAN_WORDS = 2048;              // bitmap words per compaction block
constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr uint64_t PENDING_BIT = 1ull << 63;       // two-word keys: high word claimed
constexpr uint32_t MAX_PROBE = 1u << 16;           // exact-table probe bound

// A string of S: a maximal N-free run of one genome, of length >= k.
struct DString {
    uint64_t gstart;  // global base index of its first base
    uint64_t gend;    // one past its last base
    uint32_t genome;
    uint32_t pad;
};

// Device counters of one run.
struct Counters {
    unsigned long long candidates;     // |C1|
    unsigned long long bloom_popcount;
    unsigned long long fill_atomics;   // filter atomicOr issued
    unsigned long long query_probes;   // filter words loaded by the query
    // second-pass fields, cleared before every table attempt
    unsigned long long junctions;      // |J|
    unsigned long long table_keys;     // keys claimed in the exact table
    unsigned long long overflow;       // probe bound or spin bound hit
    unsigned long long missing;        // candidate k-mers not found (must stay 0)
    unsigned long long table_probes;   // slots visited by record + decision
    unsigned long long pad[3];
};
constexpr uint32_t PASS2_COUNTERS = 5;  // junctions .. table_probes

struct SeqArgs {
    const uint64_t *seq;       // packed input as 64-bit words
    uint64_t seq_words;
    const DString *strings;
    uint32_t n_strings;
    uint32_t k;
    uint64_t n_tiles;
    uint32_t single;           // ordinary graph only (no reverse complements)
    uint32_t pad;
    const uint32_t *tile_order;        // tiles grouped per XCD, slab by slab
    uint64_t xcd_start[NXCD + 1];      // tile_order range of each XCD
};

enum KernelId { K_FILL = 0, K_QUERY = 1, K_RECORD = 2, K_DECIDE = 3, K_COUNT = 4 };

struct SentArgs {
    const void *sorted;        // normalised sentinel k-mers, ascending (W words each)
    uint32_t n;
    uint32_t pf_log2;          // prefilter size, log2 bits
    const uint32_t *prefilter;
};

struct BloomArgs {
    uint32_t *words;           // bit i: bit (i & 31) of words[i >> 5]
    uint64_t mask;             // bits - 1 (bits a power of two)
    uint32_t h;                // hash functions
    uint32_t blocked;          // blocked layout: 64-bit blocks keyed by the middle (k-1)-mer
};

// Exact-table layouts:
//   packed (k <= 27): one 64-bit word per slot, key << 8 | in/out mask
//   split  (k <= 31): key words + 8-bit masks packed 4 per 32-bit word
//   wide   (k <= 63): low and high key words + masks
struct TableArgs {
    unsigned long long *keys;     // slot words (packed) / key or low key words
    unsigned long long *keys_hi;  // high key words (wide), else null
    uint32_t *masks;              // split and wide layouts
    uint64_t capmask;             // capacity - 1
    uint32_t packed;
    uint32_t pad;
};
constexpr uint32_t PACKED_MAX_K = 27;  // 2k + 8 <= 62 bits

struct OutArgs {
    uint64_t *pos;             // genome coordinate per junction
    uint64_t *vertex;          // W words per junction
    uint8_t *strand;
    uint32_t *string_of;       // string index per junction (scratch)
    uint64_t *joff;            // n_genomes + 1
    void *edges;               // tp_edge per edge
    const uint64_t *gbase;     // per genome
    uint32_t n_genomes;
    uint32_t pad;
};

// -------------------------------------------------------------- launchers
// Resident workgroups per CU of a tile kernel (sizes its persistent grid):
// pass1_occupancy for K_FILL / K_QUERY, pass2_occupancy for K_RECORD / K_DECIDE.
hipError_t pass1_occupancy(KernelId which, int W, bool blocked, int *blocks_per_cu);
hipError_t pass2_occupancy(KernelId which, int W, int *blocks_per_cu);
hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);

// a0: normalised first/last k-mer of every string, sorted; sentinel prefilter.
hipError_t launch_sentinels(int W, const SeqArgs &a, void *raw, void *sorted,
                            uint32_t *prefilter, uint32_t pf_log2, hipStream_t s);
// a1: insert every normalised (k+1)-mer into the Bloom filter.
hipError_t launch_fill(int W, const SeqArgs &a, const BloomArgs &f, Counters *cnt, uint32_t grid,
                       hipStream_t s);
// a2: Bloom-queried neighbourhood of every k-mer position -> C1 bitmap,
// candidate count and distinct-count sketch of candidate k-mers.
hipError_t launch_query(int W, const SeqArgs &a, const BloomArgs &f, const SentArgs &sa,
                        uint64_t *c1, Counters *cnt, uint32_t *hll, uint32_t grid,
                        hipStream_t s);
hipError_t launch_popcount(const uint32_t *words, uint64_t n, Counters *cnt, hipStream_t s);
// a3: exact in/out edge masks of every candidate k-mer.
hipError_t launch_table_clear(int W, const TableArgs &t, hipStream_t s);
hipError_t launch_record(int W, const SeqArgs &a, const uint64_t *c1, const TableArgs &t,
                         Counters *cnt, uint32_t grid, hipStream_t s);
// a4: junction decision for every candidate -> J bitmap and count.
hipError_t launch_decide(int W, const SeqArgs &a, const SentArgs &sa, const uint64_t *c1,
                         const TableArgs &t, uint64_t *jbits, Counters *cnt, uint32_t grid,
                         hipStream_t s);
// a5: ordered compaction of J and compacted edges.
hipError_t launch_compact(int W, const SeqArgs &a, const uint64_t *jbits, uint64_t nwords,
                          uint32_t *blockcnt, uint64_t *blockoff, const OutArgs &o,
                          uint64_t n_junctions, hipStream_t s);

}  // namespace tp
