/*
 * twopaco.h -- C ABI of the MI355X (gfx950) TwoPaCo junction-finding library.
 *
 * Computes, for a set S of genomes and an integer k, the junction positions
 * J(S,k) of the comprehensive de Bruijn graph (Preliminaries section of
 * Minkin, Pham & Medvedev, arXiv 1602.05856) and the edges of the compacted
 * graph, which join consecutive junctions of one string (Reduction section,
 * Observation 1).  The method is Algorithm 2 (Filter-Junctions-Two-Pass) with
 * one round: a Bloom-filter pass that leaves a candidate superset C1, then an
 * exact pass over the candidates only.  k-mers are handled in normalised form
 * (the lexicographically smaller of a k-mer and its reverse complement), as
 * the reverse-complement paragraph of the Single Round section prescribes.
 *
 * Conventions shared by every entry point
 *   - Bases: A=0, C=1, G=2, T=3, packed 2 bits per base, base j of a genome in
 *     byte j>>2 at bits 2*(j&3).  N bases are listed as (start, length) runs;
 *     their packed bits are ignored.  A string of S is a maximal N-free run.
 *   - Positions are 0-based k-mer starts in genome coordinates.
 *   - A k-mer value is sum_t base[t] * 4^(k-1-t) (first base most
 *     significant), stored in W = 1 (k <= 31), W = 2 (32 <= k <= 63) or W = 4
 *     (64 <= k <= 127) 64-bit words, low word first.  Its normalised form is the smaller value of the
 *     k-mer and its reverse complement; strand 0 means the k-mer as read is
 *     its normalised form.
 *   - Status: every function returning int returns TP_OK or a negative TP_E*
 *     code and never throws.  twopaco_last_error() gives the calling thread's
 *     message for the last failure.  On failure no output is produced
 *     (*out stays NULL) and inputs are never modified.
 *   - Validation (TP_EINVAL): 1 <= k <= 127; bloom_bits a power of two with
 *     2^5 (2^6 for the blocked filter) <= bloom_bits <= 2^40 (the paper's implementation uses power-of-two
 *     filter sizes, Results section, Table 5 caption); 1 <= hash_count <= 16;
 *     N runs sorted, disjoint, non-empty and inside the genome; a packed
 *     pointer may be NULL only for a genome of 0 bases.
 *   - Device pointers are HIP device memory of the current device; a stream
 *     argument is a hipStream_t passed as void* (NULL = default stream).
 *
 * Thread safety: distinct plans may be used from distinct threads; one plan
 * must not be used concurrently.
 */
#ifndef TWOPACO_H
#define TWOPACO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TP_OK 0
#define TP_EINVAL (-1)     /* bad argument                                    */
#define TP_ENOMEM (-2)     /* host or device allocation failed                */
#define TP_EOVERFLOW (-3)  /* exact table could not be sized within limits   */
#define TP_EDEVICE (-4)    /* a HIP call failed (message has the HIP error)   */
#define TP_ESTATE (-5)     /* call out of order (e.g. outputs before a run)   */
#define TP_ETIMEOUT (-6)   /* a wait ended before the job finished           */
#define TP_EPENDING (-7)   /* tp_server_poll: the job has not finished yet   */

/* Flags. */
#define TP_FLAG_SINGLE_STRAND 1u /* ordinary graph G(S,k) of the Preliminaries
                                    section instead of G(S) u G(S-bar)        */
#define TP_FLAG_PASS1_ONLY 2u    /* partially compacted graph (Conclusion
                                    section): skip the second pass and report
                                    the first-pass candidates as junctions    */
#define TP_FLAG_BLOCKED_FILTER 4u /* first-pass Bloom filter with all h bits of
                                    a (k+1)-mer x.m.y in one 64-bit block
                                    chosen by its normalised middle (k-1)-mer m
                                    (needs bloom_bits >= 64); same junctions,
                                    one random block access per position
                                    instead of h for the fill and about
                                    6(1 + rho + ...) for the query            */

/* One genome, host memory, borrowed for the duration of the call. */
typedef struct {
    const uint8_t *packed;  /* ceil(n_bases/4) bytes, 2-bit packed            */
    uint64_t n_bases;       /* length including N bases                       */
    const uint64_t *n_runs; /* n_nruns (start, length) pairs, or NULL         */
    uint64_t n_nruns;
} tp_genome;

/* An edge of the compacted graph: the k-mers at from_pos and to_pos are
 * consecutive junctions of one string of genome `genome`. */
typedef struct {
    uint32_t genome;
    uint32_t flags; /* reserved, 0 */
    uint64_t from_pos;
    uint64_t to_pos;
} tp_edge;

/* Counters of one run (the marks-per-pass figures of Table 4 among them). */
typedef struct {
    uint64_t positions;       /* k-mer positions over all strings            */
    uint64_t candidates;      /* |C1|: positions marked after the first pass */
    uint64_t junctions;       /* |J|: positions marked after the second pass */
    uint64_t edges;           /* compacted edges                             */
    uint64_t bloom_popcount;  /* set bits of the first-pass filter           */
    uint64_t table_capacity;  /* slots of the exact table (the largest over
                                 rounds; 4096 spare slots per set included) */
    uint64_t table_keys;      /* distinct candidate k-mers in the table      */
    uint64_t distinct_estimate; /* sketch estimate used to size the table    */
    uint32_t table_attempts;  /* 1 + number of regrow-and-retry rounds       */
    uint32_t sentinels;       /* sentinel k-mers (2 per string of length >= k) */
    uint64_t edge_positions;  /* (k+1)-mer positions (filter inserts)        */
    uint64_t fill_atomics;    /* filter atomicOr issued (bit found clear)    */
    uint64_t query_probes;    /* filter words loaded by the query            */
    uint64_t table_probes;    /* table slots visited by record + decision    */
    /* Device times (HIP events on the run's stream), milliseconds. */
    float ms_sentinels;       /* sentinel set                                */
    float ms_fill;            /* Bloom fill kernel                           */
    float ms_query;           /* Bloom query kernel (+ filter popcount)      */
    float ms_record;          /* exact record (last attempt; its table clear
                                 counts in ms_pass2 only)                   */
    float ms_decide;          /* decision kernel (last attempt)              */
    float ms_pass1;           /* sentinels + fill + query                    */
    float ms_pass2;           /* all table attempts: clear, record, decide   */
    float ms_compact;         /* ordered compaction + edges                  */
    float ms_total;           /* whole run including host waits             */
    uint32_t rounds;          /* rounds (k-mer classes) the run took: the
                                 plan's, or more when tp_config.table_budget
                                 made it split the exact table              */
    uint32_t fill_chunks;     /* chunks the binned fill took per round; 0 =
                                 atomic fill (tp_config.fill_binned)         */
    uint32_t record_passes;   /* passes the binned record took (last table
                                 attempt); 0 = direct record
                                 (tp_config.record_binned)                   */
    uint32_t reserved;        /* 0 */
} tp_stats;

/* Host result, owned by the library (one page-locked block, reused by the
 * library after twopaco_result_free); free with twopaco_result_free only. */
typedef struct {
    uint32_t n_genomes;
    uint32_t kmer_words;            /* W                                        */
    uint32_t k;
    uint32_t flags;
    uint64_t n_junctions;
    const uint64_t *junction_offset; /* n_genomes+1 prefix offsets              */
    const uint64_t *junction_pos;    /* ascending within each genome            */
    const uint64_t *vertex;          /* kmer_words words per junction           */
    const uint8_t *strand;           /* one byte per junction                   */
    uint64_t n_edges;
    const tp_edge *edges;            /* genome-major, ascending from_pos        */
    tp_stats stats;
} tp_result;

/* ------------------------------------------------------------------ host API */

/* Whole build from host genomes to a host result: J(S,k) per genome (sorted),
 * vertex ids, strands and compacted edges.  Definition of the result:
 * Preliminaries section (junction), Reduction section (edges); method:
 * Algorithm 2 with one round.  Runs on the current HIP device. */
int twopaco_build(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                  uint64_t bloom_bits, uint32_t hash_count, tp_result **out);

/* As twopaco_build with TP_FLAG_* flags. */
int twopaco_build_ex(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                     uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                     tp_result **out);

void twopaco_result_free(tp_result *r);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *twopaco_last_error(void);

/* Filter size for a genome set at a given density: the smallest power of two
 * >= bits_per_edge * (number of (k+1)-mer positions), clamped to 2^6..2^40.
 * The positions bound the distinct edge count E, so by the false-positive
 * rate q = (1 - e^(-hE/b))^h of the Analysis section, 16 bits per position
 * and h = 4 keep q below 0.25%.  Host work only; 0 for invalid arguments
 * (N runs must be sorted and inside the genome). */
uint64_t tp_bloom_bits_for(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                           double bits_per_edge);

/* -------------------------------------------------------- device-level API */

/* A plan holds the layout of one or more independent genome sets (a batch)
 * and the device buffers of their runs.  Creating it does host work only (no
 * HIP call), so it can be validated without a GPU.  Genomes supply lengths
 * and N runs; packed pointers are not read here.  tp_plan_create makes a
 * batch of one set. */
typedef struct tp_plan tp_plan;

int tp_plan_create(const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                   uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                   tp_plan **out);
void tp_plan_destroy(tp_plan *p);

/* One genome set of a batch: its own S, filter size b and, at run time, its
 * own Bloom filter, sentinel set, exact table, junctions and edges (the
 * result of every set equals that of a plan holding it alone).  k, h and
 * flags are shared by the batch.  Genome indices of a batch are global:
 * set s owns genomes tp_plan_set_first_genome(s) .. + n_genomes - 1, in
 * order. */
typedef struct {
    const tp_genome *genomes;
    uint32_t n_genomes;
    uint32_t reserved;      /* 0 */
    uint64_t bloom_bits;    /* this set's filter size (validated as above),
                               or 0: sized by the plan at
                               tp_config.bloom_bits_per_edge bits per
                               (k+1)-mer position, as tp_bloom_bits_for
                               does (see tp_plan_set_bloom_bits)          */
} tp_set;

/* A batch of n_sets >= 1 sets: every phase of a run is one launch over all
 * sets' tiles (each tile reads its set's descriptor), and the host waits
 * three times per batch instead of three times per set.  Batches of several
 * sets size each exact table from its set's candidate count (no sketch). */
int tp_batch_create(const tp_set *sets, uint32_t n_sets, uint32_t k, uint32_t hash_count,
                    uint32_t flags, tp_plan **out);
uint32_t tp_plan_sets(const tp_plan *p);
uint32_t tp_plan_set_first_genome(const tp_plan *p, uint32_t set);
/* 32-bit words of the filter pool, and the first word of a set's filter in
 * it (tp_device_outputs.bloom points at the pool). */
uint64_t tp_plan_bloom_words(const tp_plan *p);
uint64_t tp_plan_set_bloom_offset(const tp_plan *p, uint32_t set);
/* A set's filter size in bits: the one it was given, or for a set given 0
 * the size the plan chose under its current configuration (0 for a bad
 * argument). */
uint64_t tp_plan_set_bloom_bits(const tp_plan *p, uint32_t set);

/* Device input layout: all genomes in one buffer of tp_plan_input_bytes()
 * bytes, genome g starting at byte tp_plan_genome_offset(g) (a multiple of
 * 64), zero elsewhere.  Its 2-bit base index (byte offset * 4 + base) is the
 * "global base index" used by the bitmaps below. */
uint64_t tp_plan_input_bytes(const tp_plan *p);
uint64_t tp_plan_genome_offset(const tp_plan *p, uint32_t genome);
/* 64-bit words of a position bitmap (bit i of word w is global base index
 * 64*w + i). */
uint64_t tp_plan_bitmap_words(const tp_plan *p);
/* Number of strings (contigs of length >= k). */
uint64_t tp_plan_strings(const tp_plan *p);

/* Copy the host genomes into a caller-owned device buffer of
 * tp_plan_input_bytes() bytes (asynchronous on `stream`; host buffers must
 * stay valid until the stream reaches this point). */
int tp_plan_upload(tp_plan *p, const tp_genome *genomes, uint8_t *d_input, void *stream);
/* The same for a batch: sets[s] must list the genomes of set s in order. */
int tp_batch_upload(tp_plan *p, const tp_set *sets, uint8_t *d_input, void *stream);

/* Algorithm 3 (Multiple Rounds section): split the normalised k-mers into
 * `rounds` classes and run Algorithm 2 once per class, so each round's filter
 * holds only the edges next to its class's k-mers and each round's exact
 * table only its candidates (the peak table shrinks about `rounds`-fold).
 * Classes are runs of 1024 hash subranges formed by the section's greedy
 * scan over per-subrange counters of (k+1)-mer occurrences, computed per set
 * on the device.  Junctions, vertices and edges are those of one round; the
 * candidate bitmap (tp_debug_candidates, tp_device_outputs.candidates) is
 * the union of the rounds' first-pass marks, tp_debug_bloom the last round's
 * filter, and candidates / bloom_popcount / table_keys in tp_stats are sums
 * over rounds.  1 <= rounds <= 64; default 1; takes effect at the next
 * tp_run.  tp_plan_class_bounds gives a set's rounds + 1 subrange bounds
 * after a run. */
int tp_plan_set_rounds(tp_plan *p, uint32_t rounds);
uint32_t tp_plan_rounds(const tp_plan *p);
int tp_plan_class_bounds(const tp_plan *p, uint32_t set, uint32_t *bounds, uint32_t n);

/* Runtime knobs of a plan.  They change speed only, never results (every
 * output is bit-identical under any setting). */
typedef struct {
    uint32_t wg_per_cu[4]; /* resident workgroups per CU of the persistent
                              fill, query, record and decision kernels;
                              0 = as many as fit                            */
    uint32_t tile_order;   /* first pass: 0 = homologous tiles of a set's
                              genomes as slabs, slabs round-robin over the
                              8 XCDs, set by set; 1 = memory order cut into
                              8 contiguous ranges, one per XCD              */
    float table_load;      /* exact-table sizing: slots = keys / table_load
                              rounded up to a multiple of 64, keys
                              estimated by a sketch (one set) or bounded by
                              the candidate count (batches); in [0.05, 16].
                              A table that overflows is doubled and the pass
                              repeated.                                     */
    uint32_t graphs;       /* 1: the multi-launch sequences of a run (the
                              sentinel kernels and zeroing before the fill,
                              the counter and table clearing before record,
                              the whole compaction) are captured once as
                              HIP graphs on a private stream and replayed on
                              the run's stream; captured again whenever a
                              buffer, size or argument changes.  The timed
                              kernels stay direct launches between their
                              events.  Single-round plans only (ignored with
                              rounds > 1).  0 = every launch direct.        */
    uint32_t pass2_slabs;  /* second-pass tile order: bit 0 record, bit 1
                              decision; set = the first pass's order
                              (homologous tiles at the same time, sharing
                              table lines in L2), clear = memory order; bit
                              2 = record in runs of 8 consecutive entries of
                              the first pass's order per workgroup visit
                              (overrides bit 0)                              */
    uint32_t fill_dedup;   /* blocked filter, fill: 1 = each workgroup walks
                              runs of 8 consecutive first-pass tiles
                              (homologous regions) and skips an edge whose
                              filter bits it has already sent; 0 = off      */
    uint32_t table_shape;  /* exact-table capacity: 1 = a power of two (home
                              slot = low hash bits, probes wrap); 2 = any
                              size: whole blocks of 8192 slots (one block of
                              a power of two up to 8192 slots), the home
                              block by a 32-bit multiply, probes wrapping
                              within it (rounds up by less than 8192 slots);
                              0 = a power of two unless rounding up would
                              leave more than 4 GiB of slots unused over the
                              run's sets                                   */
    uint32_t chunk_tiles;  /* chunk size of the persistent tile walks: a
                              workgroup takes this many consecutive tiles
                              (2048 positions each) of its walk per visit,
                              1..64                                          */
    uint32_t fill_binned;  /* blocked filter, fill: 0 = binned when some
                              set's filter is at least 1 GiB, else atomic;
                              1 = atomic (each edge's block loaded, then an
                              atomicOr for bits still clear, in HBM); 2 =
                              binned: per chunk of positions, every
                              edge's filter effect is written as an
                              8-byte item, the items partitioned by 64 KiB
                              region of the pool in two streaming passes,
                              and each region's items ORed into the region
                              in LDS.  Same filter bits either way.  Binned
                              needs 16 bytes per chunk position of scratch,
                              held in the exact table's key buffer (the
                              table is not live during the fill), and a
                              pool of at most 32 GiB (else atomic).  Runs
                              on caller memory (tp_run_ws, tp_run_noalloc)
                              always fill atomically.                        */
    uint32_t bin_chunk_tiles; /* binned fill: tiles (2048 positions each)
                              per chunk, 1..2^20; 0 = 2^20 (2^31
                              positions), or more, up to 2^22, when the
                              key buffer of an earlier run's table holds
                              them.  Each chunk rereads the filter once.   */
    uint32_t bloom_bits_per_edge; /* sets created with bloom_bits 0: filter
                              bits per (k+1)-mer position, rounded up to a
                              power of two (2^6..2^40); 0 = 16, else
                              1..256.  Changing it re-lays out the filter
                              pool (host work).  The junctions do not
                              depend on it (the second pass is exact); the
                              candidate count, and so the second pass's
                              work, does.                                   */
    uint32_t tile_queue;   /* 1: the fill, query, record and decision take
                              their chunks of tiles from device counters
                              (one per XCD share of the tile order, claimed
                              with an atomic add; a workgroup whose share is
                              exhausted takes chunks of the other shares),
                              so the last chunks go to whichever workgroups
                              are free (a kernel with fewer than 4 tiles
                              per workgroup keeps the static schedule); 0 =
                              a static schedule (every grid-th chunk)      */
    uint32_t record_binned; /* exact record of a one-set plan with k <= 27
                              whose table is any-size (table_shape) or at
                              most 8192 slots: 0 = binned when the table is
                              at least 1 GiB and its scratch takes at most 2
                              passes, else direct (each pass walks all
                              candidates again); 1 = direct (random
                              atomics into the table); 2 = binned whenever
                              scratch is found.  Binned: a lookup never
                              leaves the 8192-slot block of its home slot,
                              so per pass (a range of blocks) every
                              candidate of that range becomes an 8-byte
                              item, the items are partitioned by block in
                              two streaming passes and each block is built
                              in LDS and written out whole.  Same keys and
                              edge bits, so the same junctions.  Scratch: 16
                              bytes per item of a pass, in the last run's
                              edge array (dead until the compaction) or in a
                              buffer of its own when the device has room
                              (1 GiB left free; kept by the plan until its
                              outputs must grow); else, and for plans of a
                              server, the record runs directly, as it does
                              on caller memory (tp_run_ws, tp_run_noalloc).
                              A pass holds at most 2^19 blocks (32 GiB of
                              table).  The passes taken are in
                              tp_stats.record_passes.                        */
    uint64_t table_budget; /* exact-table budget in bytes (0: none).  A
                              one-round run whose exact table, sized after
                              the first pass, would exceed it is redone as
                              Algorithm 3 with enough rounds (k-mer classes)
                              that each round's table fits, about; the
                              junctions are those of one round.  The rounds
                              taken are in tp_stats.rounds.                  */
    uint32_t record_passes; /* binned record: at least this many passes
                              (0 = as the scratch needs), 0..64              */
    uint32_t reserved;     /* 0 */
} tp_config;

/* Defaults: all workgroups that fit for fill and query, 6 per CU for record
 * and decision, order 0, table_load 0.7 for one set and 0.5 for batches,
 * graphs 0, pass2_slabs 2 (decision in first-pass order), fill_dedup 1
 * (ignored with the standard filter), table_shape 0, chunk_tiles 1,
 * fill_binned 0, bin_chunk_tiles 0, bloom_bits_per_edge 0 (16),
 * tile_queue 1, record_binned 0, table_budget 0, record_passes 0.  tp_plan_set_config fails with TP_EINVAL outside the
 * ranges above and leaves the plan unchanged. */
int tp_plan_get_config(const tp_plan *p, tp_config *out);
int tp_plan_set_config(tp_plan *p, const tp_config *cfg);

/* Autotuner: times the plan's kernels on its own input under candidate
 * configurations (about 48 runs of tp_run; 6 more when some set's filter is
 * auto-sized, whose density it picks among 8, 16 and 32 bits per (k+1)-mer
 * on the whole run; with the blocked filter it also picks the atomic or the
 * binned fill), keeps the fastest per knob and applies it.  With a
 * cache file, results are keyed by device, k-mer words, flags, position
 * count (power-of-two bucket), set count (bucket) and whether some filter is
 * auto-sized; a
 * cached entry is applied without any run, and new entries are added to the
 * file (rewritten whole; NULL = no cache).  The plan's outputs afterwards are
 * those of its last run. */
int tp_autotune(tp_plan *p, const uint8_t *d_input, void *stream, const char *cache_path,
                tp_config *out);

/* Run the whole path on a device input laid out as above: sentinels, Bloom
 * fill, Bloom query (C1), exact-table record, decision (J), ordered
 * compaction and edges.  The device input is borrowed; device outputs stay
 * owned by the plan until the next run or tp_plan_destroy.  The call waits
 * on `stream` at three points (candidate count, table check, junction count)
 * and returns when the outputs are complete.  Device buffers are kept across
 * runs; when one cannot grow, the buffers dead at that point are freed and
 * the allocation tried once more (the previous run's outputs before the
 * exact table, the exact table before the outputs), so a run whose table and
 * outputs do not fit HBM together still completes, at the cost of
 * reallocating them on every run.  TP_ENOMEM when even that fails. */
int tp_run(tp_plan *p, const uint8_t *d_input, void *stream);

/* Counters of the last run, whole batch. */
int tp_get_stats(const tp_plan *p, tp_stats *out);
/* Counters of one set of the last run: positions, candidates, junctions,
 * edges, bloom_popcount, table_capacity, table_keys, sentinels and
 * edge_positions are the set's; probes, estimate, attempts and device times
 * are the batch's. */
int tp_get_set_stats(const tp_plan *p, uint32_t set, tp_stats *out);

/* Device views of the last run's outputs (owned by the plan). */
typedef struct {
    uint64_t n_junctions;
    uint64_t *junction_offset; /* n_genomes+1                                  */
    uint64_t *junction_pos;    /* n_junctions                                  */
    uint64_t *vertex;          /* n_junctions * W                              */
    uint8_t *strand;           /* n_junctions                                  */
    uint64_t n_edges;
    tp_edge *edges;            /* n_edges                                      */
    uint64_t *candidates;      /* C1 bitmap, tp_plan_bitmap_words() words      */
    uint64_t *junction_bits;   /* J bitmap, same layout                        */
    uint32_t *bloom;           /* filter pool, tp_plan_bloom_words() words     */
} tp_device_outputs;

int tp_get_device_outputs(const tp_plan *p, tp_device_outputs *out);

/* Copy the last run's outputs into a new host result (waits on `stream`):
 * tp_download all genomes of the batch, tp_download_set those of one set,
 * with genome indices (junction_offset, edges) relative to the set's first
 * genome and the set's counters in stats. */
int tp_download(const tp_plan *p, void *stream, tp_result **out);
int tp_download_set(const tp_plan *p, uint32_t set, void *stream, tp_result **out);

/* Debug taps used by parity tests: copy a set's first-pass filter words
 * (its bloom_bits/32 uint32; tp_debug_bloom: set 0) or the candidate bitmap
 * (tp_plan_bitmap_words() uint64) of the last run to host memory.  Wait on
 * the device. */
int tp_debug_bloom(const tp_plan *p, uint32_t *host_words, uint64_t n_words);
int tp_debug_set_bloom(const tp_plan *p, uint32_t set, uint32_t *host_words, uint64_t n_words);
int tp_debug_candidates(const tp_plan *p, uint64_t *host_words, uint64_t n_words);

/* Whole build of a batch of independent genome sets from host memory to one
 * host result per set (as tp_download_set gives them: genome indices
 * relative to the set, the set's own counters): tp_batch_create, upload,
 * tp_run and one download per set.  results[s] receives set s's result (free
 * each with twopaco_result_free); on failure every results[s] is NULL.  The
 * result of every set equals that of a build of the set alone (Algorithm 2
 * run on each set's S). */
int tp_build_batch(const tp_set *sets, uint32_t n_sets, uint32_t k, uint32_t hash_count,
                   uint32_t flags, tp_result **results);

/* Debug tap used by parity tests: the exact second-pass table of one set
 * after the last run (the last round's table with rounds > 1).  Every
 * occupied slot gives one entry: the normalised candidate k-mer (kmer_words
 * words per entry, low word first, into keys) and its edge mask (into masks):
 * bits 0-3 the bases c with c.v an edge of the comprehensive graph, bits 4-7
 * the bases c with v.c an edge, v in normalised orientation (the per-vertex
 * form of the edge table of Algorithm 2's second pass).  Entries come in slot
 * order; *n_out receives their number.  With cap smaller than that number
 * nothing is written and TP_EINVAL is returned (*n_out still set).  Waits on
 * the device.  TP_ESTATE without a completed run, in pass-1-only mode, or when
 * the run released its table to fit its outputs. */
int tp_debug_table(const tp_plan *p, uint32_t set, uint64_t *keys, uint8_t *masks, uint64_t cap,
                   uint64_t *n_out);

/* ------------------------------------------- caller-owned memory (workspace) */

/* The whole path on a device input, with every device buffer owned by the
 * caller: a workspace (filters, candidate and junction bitmaps, sentinels,
 * exact tables, counters, layout tables) and an output buffer (counts and the
 * result arrays).  The run is a sequence of kernel launches on the caller's
 * stream with no host wait and no allocation, so a caller may capture it in
 * a HIP graph and replay it.
 *
 * Exact tables cannot grow without a host wait, so they are sized from a
 * bound the caller states: each set's distinct candidate k-mers are at most
 * key_fraction times its k-mer positions (1 is always enough; the bacterial
 * workloads need about 0.05-0.3), at the plan's table_load.  Outputs are
 * sized for at most junction_fraction times the plan's k-mer positions
 * junctions (1 is always enough).  When a bound does not hold, the run
 * reports it in the counts' status and its outputs are not valid (table) or
 * truncated (outputs); no access leaves the buffers.
 *
 * Output buffer (tp_ws_layout offsets, bytes from its start):
 *   counts      one tp_ws_counts
 *   joff        uint64[n_genomes + 1]: junction offsets per genome
 *   pos         uint64[max_junctions]: ascending within each genome
 *   vertex      uint64[max_junctions * kmer_words]
 *   strand      uint8[max_junctions]
 *   edges       tp_edge[max_edges]: genome-major, ascending from_pos
 * Workspace (offsets for inspection): the candidate bitmap C1 (the union over
 * rounds), the junction bitmap J (tp_plan_bitmap_words() words each), the
 * filter pool (tp_plan_bloom_words() words; the last round's filter) and one
 * tp_ws_set_counters per set. */
typedef struct {
    uint64_t status;          /* 0: complete; bit 0: a set's candidate k-mers
                                 overflowed its table (outputs not valid);
                                 bit 1: more junctions than max_junctions
                                 (outputs truncated); bit 2: internal error */
    uint64_t positions;       /* k-mer positions over all strings            */
    uint64_t candidates;      /* |C1| (sum over rounds)                      */
    uint64_t junctions;       /* |J|                                         */
    uint64_t edges;           /* compacted edges                             */
    uint64_t table_keys;      /* distinct candidate k-mers (sum over rounds) */
    uint64_t bloom_popcount;  /* filter bits set (sum over rounds)           */
    uint64_t reserved[9];
} tp_ws_counts;

#define TP_WS_TABLE_OVERFLOW 1u
#define TP_WS_OUTPUT_OVERFLOW 2u
#define TP_WS_INTERNAL 4u

typedef struct {
    uint64_t candidates, bloom_popcount, junctions, table_keys, overflow, reserved[3];
} tp_ws_set_counters;

typedef struct {
    uint64_t workspace_bytes;     /* size of the workspace buffer             */
    uint64_t output_bytes;        /* size of the output buffer                */
    uint64_t max_junctions, max_edges;
    uint64_t table_slots;         /* all sets' tables, spare tails included   */
    uint32_t kmer_words, rounds;
    /* offsets into the output buffer */
    uint64_t off_counts, off_joff, off_pos, off_vertex, off_strand, off_edges;
    /* offsets into the workspace */
    uint64_t ws_off_candidates, ws_off_junction_bits, ws_off_bloom, ws_off_set_counters;
} tp_ws_layout;

/* Lay out the workspace and output buffer of a plan for the given bounds
 * (0 < key_fraction <= 1, 0 < junction_fraction <= 1) under its current
 * rounds, flags and table_load.  Host work only.  A later tp_plan_set_rounds
 * or tp_plan_set_config invalidates the layout (tp_run_ws then fails with
 * TP_ESTATE until it is laid out and prepared again). */
int tp_plan_workspace_layout(tp_plan *p, double key_fraction, double junction_fraction,
                             tp_ws_layout *out);
/* Workspace bytes of the plan's current layout (0 when it has none). */
uint64_t tp_plan_workspace_bytes(const tp_plan *p);

/* Write the plan's layout tables (strings, tiles, set descriptors) into a
 * workspace of tp_plan_workspace_bytes() bytes, asynchronously on `stream`
 * (the plan keeps the host copies alive).  Needed once per workspace before
 * tp_run_ws; the plan remembers the last workspace it prepared. */
int tp_plan_prepare_workspace(tp_plan *p, void *d_workspace, void *stream);

/* Run the whole path (sentinels, Bloom fill, Bloom query, exact record,
 * decision, ordered compaction and edges; Algorithm 2, or Algorithm 3 with
 * the plan's rounds) on a device input laid out as for tp_run, using the
 * prepared workspace and writing the output buffer.  Asynchronous: returns
 * after enqueueing on `stream`; counts and status are in the output buffer
 * once the stream reaches the end of the run.  TP_ESTATE when the workspace
 * is not the one last prepared for the plan's current layout.  No timing
 * counters (tp_get_stats describes tp_run only). */
int tp_run_ws(tp_plan *p, const uint8_t *d_input, void *d_workspace, void *d_outputs,
              void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tp_run_ws
 * with the library's own fixed workspace instead of a caller workspace.  The
 * plan needs a current workspace layout (tp_plan_workspace_layout) of at most
 * TP_NOALLOC_WORKSPACE_MAX bytes, else TP_EINVAL (nothing runs); the caller
 * passes the input and an output buffer of the layout's output_bytes.  The
 * call rewrites the fixed workspace's layout tables (asynchronous copies
 * from the plan's host memory) and enqueues the run; it allocates nothing.
 * The fixed workspace is one device array per GPU, held from library load
 * until the process ends and shared by every call on that GPU: calls that
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller. */
#define TP_NOALLOC_WORKSPACE_MAX (64ull << 20)
int tp_run_noalloc(tp_plan *p, const uint8_t *d_input, void *d_outputs, void *stream);

/* ------------------------------------------------------- measurement aid */

/* Not part of the method: the rate at which the device serves random 8-byte
 * accesses into a buffer of `bytes` bytes (the access pattern of the Bloom
 * fill and query and of the exact-table record and decision, without their
 * arithmetic), for the roofline of those kernels.  Makes about `accesses`
 * uniformly random accesses (mode 0: relaxed device-scope loads; mode 1:
 * atomic ORs of one bit, the fill's read-modify-write), addresses drawn
 * from a counter-based hash of `seed`, and XORs every loaded word into
 * *d_checksum (device memory, 8 bytes) so that no access can be dropped.
 * Asynchronous on `stream`; *accesses_done (host) receives the exact
 * number of accesses.  Mode 1 modifies the buffer. */
int tp_bench_random_access(void *d_buf, uint64_t bytes, uint64_t accesses, uint32_t mode,
                           uint64_t seed, uint64_t *d_checksum, void *stream,
                           uint64_t *accesses_done);

/* ------------------------------------------------------------- serving */

/* A server builds graphs for jobs submitted at any time, on the device that
 * is current when it is created.  Worker threads each own a stream and a
 * reusable plan whose device buffers persist from job to job (a warm server
 * allocates no device memory).  Admission: a job starts when the bytes held
 * or reserved by all workers plus its estimate fit hbm_budget; jobs start in
 * arrival order, except that express workers (the last express_workers of
 * them) take only jobs of at most batch_max_bases bases -- the oldest such
 * job -- so small jobs need not wait behind large ones; with express_cus
 * set, small jobs go to the express workers only.  Continuous batching: a
 * worker that takes a job of at most
 * batch_max_bases bases also takes the queued jobs behind it with the same
 * k, hash_count and flags (each at most batch_max_bases, together at most
 * batch_total_bases, at most max_batch jobs) and runs them as one batched
 * plan.  Every job's result is the one a build of it alone gives.  The
 * serving pattern itself is not in the paper, whose method each job runs. */
typedef struct tp_server tp_server;

typedef struct {
    uint64_t hbm_budget;        /* device bytes all workers may hold          */
    uint32_t workers;           /* worker threads and streams, 1..16          */
    uint32_t max_batch;         /* jobs per batched plan, >= 1 (1 = none)     */
    uint64_t batch_max_bases;   /* largest job that is batched                */
    uint64_t batch_total_bases; /* bases per batched plan at most             */
    uint32_t wg_per_cu;         /* resident workgroups per CU of every job's
                                   tile kernels (tp_config), so concurrent
                                   jobs share the CUs; 0 = all that fit       */
    uint32_t express_workers;   /* of the workers, how many take only jobs of
                                   at most batch_max_bases bases; < workers   */
    uint32_t express_cus;       /* CUs kept for the express workers' kernels
                                   (their streams run on these CUs only, the
                                   other workers' on the rest, and only the
                                   express workers take small jobs), so a
                                   small job never waits for CU room behind
                                   a large one; 0 = all workers share every
                                   CU                                         */
    uint32_t table_budget_mib;  /* cap on any job's exact tables, MiB (0 =
                                   none): each job's plan runs with this
                                   tp_config.table_budget, so a job whose
                                   table would exceed it is built in enough
                                   rounds (Algorithm 3, Multiple Rounds
                                   section) that each round's table fits,
                                   with the same junctions                    */
} tp_server_opts;

/* Times are seconds since the server was created (host steady clock). */
typedef struct {
    double submit_s, start_s, end_s;
    uint32_t batch_jobs;        /* jobs in the plan that ran it               */
    uint32_t worker;
    uint64_t bases;             /* bases of its genomes, N included           */
    float layout_ms;            /* host: laying out the plan                  */
    float upload_ms;            /* host to device copy of the batch's input   */
    float run_ms;               /* tp_run of the batch, host waits included   */
    float download_ms;          /* device to host copy of this job's result   */
} tp_job_info;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t batches;           /* plans run                                  */
    uint64_t queued, running;
    uint64_t held_bytes;        /* device bytes the workers' buffers hold     */
    uint64_t peak_held_bytes;
} tp_server_stats;

int tp_server_create(const tp_server_opts *opts, tp_server **out);
/* Validates the job as tp_plan_create does and copies its genomes (the
 * caller's buffers are free on return).  *job_id identifies it for
 * tp_server_wait. */
int tp_server_submit(tp_server *s, const tp_genome *genomes, uint32_t n_genomes, uint32_t k,
                     uint64_t bloom_bits, uint32_t hash_count, uint32_t flags,
                     uint64_t *job_id);
/* Wait for a job (timeout_ms < 0: no limit).  On TP_OK *out is its result
 * (free with twopaco_result_free; stats are the job's own counters with the
 * batch's device times) and *info its times (info may be NULL); the job is
 * then forgotten.  A failed job returns its status and is forgotten too;
 * TP_ETIMEOUT leaves it waiting.  A job too large for hbm_budget fails with
 * TP_ENOMEM. */
int tp_server_wait(tp_server *s, uint64_t job_id, int64_t timeout_ms, tp_result **out,
                   tp_job_info *info);
/* Non-blocking wait: TP_OK with the job's result and times when it has
 * finished (the job is then forgotten, as after tp_server_wait), its failure
 * status when it failed, TP_EPENDING while it is queued or running.  A job
 * may be waited for or polled from one thread at a time: a second caller
 * gets TP_ESTATE while another is waiting for it. */
int tp_server_poll(tp_server *s, uint64_t job_id, tp_result **out, tp_job_info *info);
int tp_server_get_stats(tp_server *s, tp_server_stats *out);
/* Finishes running jobs, fails queued ones with TP_ESTATE, wakes and waits
 * out callers blocked in tp_server_wait (they return TP_ESTATE), frees
 * everything.  No call may follow. */
void tp_server_destroy(tp_server *s);

#ifdef __cplusplus
}
#endif

#endif /* TWOPACO_H */
