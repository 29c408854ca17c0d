// First pass of Algorithm 2 (Filter-Junctions with E = Bloom filter) and the
// sentinel set, for gfx950.
//
//   k_sentinel_values, k_sentinel_table, k_prefilter
//                 normalised first and last k-mer of every string (the
//                 sentinel vertices of the Preliminaries section, both
//                 strands), a hash table of them per set, plus a bit
//                 prefilter
//   k_fill        loop 1 of Algorithm 1 with every position marked: every
//                 normalised (k+1)-mer goes into its set's filter (load first,
//                 atomicOr only for bits still clear)
//   k_query       loop 2 of Algorithm 1: a position stays marked when it is a
//                 string end, a sentinel k-mer, or when any of its six
//                 neighbour (k+1)-mers other than the actual predecessor and
//                 successor edge tests present (in = 1 and out = 1 fails).
//                 Writes the C1 bitmap with one wave ballot per 64 positions.
//
// Both filter layouts share the tile loop (template flag BLOCKED):
//   standard  h bits anywhere in the filter; the query probes its six
//             neighbours level by level (bit t of every neighbour still
//             possibly present, so up to six loads are in flight per lane)
//   blocked   all h bits of an edge x.m.y in the 64-bit block of its
//             normalised middle m (see MiddleKey); a position's out-edges
//             share the block of its out-middle v[1..k-1], its in-edges the
//             block of its in-middle v[0..k-2] -- the out-middle of the
//             position before, passed by a wave shuffle -- so a position
//             costs one random load.
//
// Sequence reads: each workgroup stages its tile's packed words (plus one
// word before and three after, covering predecessor, successor and the
// longest window) in LDS with coalesced 64-bit loads; lanes then extract
// their k-mer windows from LDS.
#include "device.hpp"

namespace tp {

__global__ void k_zero(uint4 *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ void k_zero_bytes(uint8_t *p, uint64_t n) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static uint32_t grid_for(uint64_t n, uint32_t cap = 8192) {
    uint64_t g = (n + BLOCK - 1) / BLOCK;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s) {
    if (bytes == 0)
        return hipSuccess;
    uint64_t n16 = bytes / 16, tail = bytes % 16;
    if (n16) {
        hipLaunchKernelGGL(k_zero, dim3(grid_for(n16)), dim3(BLOCK), 0, s, (uint4 *)p, n16);
    }
    if (tail) {
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(BLOCK), 0, s, (uint8_t *)p + n16 * 16,
                           tail);
    }
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n)), dim3(BLOCK), 0, s, p, n, v);
    return hipGetLastError();
}

// Stage the packed words of tile `tile` into w: word i of w is global word
// tile*TILE_WORDS - 1 + i (zero outside the buffer).  Base index r of w is
// global base index tile*TILE - 32 + r.
__device__ __forceinline__ void stage_tile(const SeqArgs &a, uint64_t tile, uint64_t *w) {
    int64_t w0 = (int64_t)(tile * TILE_WORDS) - 1;
    for (uint32_t i = threadIdx.x; i < STAGE_WORDS; i += blockDim.x) {
        int64_t gw = w0 + (int64_t)i;
        w[i] = (gw >= 0 && (uint64_t)gw < a.seq_words) ? a.seq[gw] : 0ull;
    }
}

// ------------------------------------------------------------ sentinels (a0)

template <class T>
__global__ void k_sentinel_values(SeqArgs a, T *out) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_strings)
        return;
    DString s = a.strings[i];
    uint64_t first = s.gstart, last = s.gend - a.k;
    T x0 = KT<T>::window(a.seq + (first >> 5), (uint32_t)(first & 31), a.k);
    T x1 = KT<T>::window(a.seq + (last >> 5), (uint32_t)(last & 31), a.k);
    out[2 * i] = norm(strands(x0, a.k), a.single != 0);
    out[2 * i + 1] = norm(strands(x1, a.k), a.single != 0);
}

// Each set's sentinel table: thread i inserts sentinel i (of string i / 2,
// hence of that string's set) by claiming a slot's claim word; a k-mer that
// another sentinel of the set has already claimed is not inserted twice.
// Lookups run in later kernels, after every value is in place.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_sentinel_table(SeqArgs a, const T *raw, uint32_t n,
                                                          T *tab, uint32_t *owner) {
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n)
        return;
    const SetDesc &d = a.sets[a.strings[i / 2].set];
    if (!d.sent_tab_log2)
        return;
    const T v = raw[i];
    const uint32_t mask = (1u << d.sent_tab_log2) - 1;
    T *t = tab + d.sent_tab_off;
    uint32_t *o = owner + d.sent_tab_off;
    uint32_t s = sent_home(v, d.sent_tab_log2);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const uint32_t prev = atomicCAS(&o[s], ~0u, i);
        if (prev == ~0u) {
            t[s] = v;
            return;
        }
        if (raw[prev] == v)
            return;  // the same k-mer, inserted by another sentinel
        s = (s + 1) & mask;
    }
}

template <class T>
__global__ void k_prefilter(const T *vals, uint32_t n, uint32_t log2bits, uint32_t *bits) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t b = prefilter_bit(vals[i], log2bits);
    atomicOr(&bits[b >> 5], 1u << (b & 31));
}

template <class T>
static hipError_t sentinels_t(const SeqArgs &a, void *raw, void *tab, uint32_t *owner,
                              uint64_t tab_slots, uint32_t *prefilter, uint32_t pf_log2,
                              hipStream_t s) {
    uint32_t n = 2 * a.n_strings;
    hipError_t e = launch_zero(prefilter, (1ull << pf_log2) / 8, s);
    if (e == hipSuccess && tab_slots) {
        e = launch_fill_u64((uint64_t *)tab, tab_slots * KT<T>::W, ~0ull, s);
        if (e == hipSuccess)
            e = launch_fill_u64((uint64_t *)owner, (tab_slots + 1) / 2, ~0ull, s);
    }
    if (e != hipSuccess || n == 0)
        return e;
    uint32_t g1 = (a.n_strings + BLOCK - 1) / BLOCK, g2 = (n + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_sentinel_values<T>, dim3(g1), dim3(BLOCK), 0, s, a, (T *)raw);
    hipLaunchKernelGGL(k_sentinel_table<T>, dim3(g2), dim3(BLOCK), 0, s, a, (const T *)raw, n,
                       (T *)tab, owner);
    hipLaunchKernelGGL(k_prefilter<T>, dim3(g2), dim3(BLOCK), 0, s, (const T *)raw, n, pf_log2,
                       prefilter);
    return hipGetLastError();
}

hipError_t launch_sentinels(int W, const SeqArgs &a, void *raw, void *tab, uint32_t *tab_owner,
                            uint64_t tab_slots, uint32_t *prefilter, uint32_t pf_log2,
                            hipStream_t s) {
    return by_width(W, [&](auto tag) {
        return sentinels_t<decltype(tag)>(a, raw, tab, tab_owner, tab_slots, prefilter, pf_log2,
                                          s);
    });
}

// ---------------------------------------------------------------- fill (a1)

// Standard layout: h words, loads issued together, atomicOr for clear bits.
template <class T>
__device__ __forceinline__ uint32_t insert_standard(const BloomArgs &f, const Strands<T> &e,
                                                    bool single) {
    const BloomHash bh = bloom_hash(norm(e, single));
    uint64_t idx[16];
    uint32_t cur[16];
#pragma unroll
    for (uint32_t t = 0; t < 16; ++t) {
        if (t < f.h) {
            idx[t] = (bh.h1 + (uint64_t)t * bh.h2) & f.mask;
            cur[t] = __hip_atomic_load(&f.words[idx[t] >> 5], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    uint32_t atomics = 0;
#pragma unroll
    for (uint32_t t = 0; t < 16; ++t) {
        if (t < f.h) {
            const uint32_t bit = 1u << (idx[t] & 31);
            if (!(cur[t] & bit)) {
                __hip_atomic_fetch_or(&f.words[idx[t] >> 5], bit, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                ++atomics;
            }
        }
    }
    return atomics;
}

// Blocked layout: one 64-bit block keyed by the edge's middle.  With a
// dedup table dd (LDS), an edge whose effect on the filter -- block, offset,
// stride and pair, which fix the bits it sets -- some lane of this workgroup
// has already sent is skipped: that lane's load and atomic complete within
// the kernel, and filter bits are only ever set.  Lanes racing on one entry
// both send.
template <class T>
__device__ __forceinline__ uint32_t insert_blocked(const BloomArgs &f, const Strands<T> &e,
                                                   uint32_t k, bool single,
                                                   unsigned long long *dd) {
    const T mid_ones = KT<T>::ones(2 * (k - 1));
    unsigned long long *blocks = (unsigned long long *)f.words;
    const uint32_t x = (uint32_t)(e.fwd >> (2 * k)), y = (uint32_t)(e.fwd & 3);
    const MiddleKey key = middle_key((T)((e.fwd >> 2) & mid_ones), (T)((e.rc >> 2) & mid_ones),
                                     single, f.mask >> 6);
    const uint32_t j = pair_index(key.orient, x, y, e.fwd <= e.rc);
    if (dd) {
        const unsigned long long id =
            (unsigned long long)key.block << 16 | key.a | key.d << 6 | j << 12;
        unsigned long long *slot = &dd[(key.block * 16 + j) & (FILL_DD - 1)];
        if (*slot == id)
            return 0;
        *slot = id;
    }
    const uint64_t m = pair_mask(key.a, key.d, j, f.h);
    const unsigned long long cur =
        __hip_atomic_load(&blocks[key.block], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((cur & m) == m)
        return 0;
    __hip_atomic_fetch_or(&blocks[key.block], (unsigned long long)m, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
    return 1;
}

template <class T, bool BLOCKED>
__global__ __launch_bounds__(BLOCK) void k_fill(SeqArgs a, BloomArgs pool, Counters *cnt) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ unsigned long long block_atomics;
    extern __shared__ unsigned long long dd_lds[];  // FILL_DD entries when deduplicating
    const uint32_t L = a.k + 1;
    const bool single = a.single != 0;
    unsigned long long *dd = BLOCKED && a.fill_dedup ? dd_lds : nullptr;
    uint32_t dd_set = ~0u;  // the set whose filter effects dd holds
    if (threadIdx.x == 0)
        block_atomics = 0;
    uint32_t my_atomics = 0;
    // with dedup, runs of homologous tiles
    RunCursor rc = run_cursor(a, dd ? (a.chunk > FILL_CHUNK ? a.chunk : FILL_CHUNK) : a.chunk);
    for (uint64_t tile; run_next(a, rc, &tile);) {
        const uint64_t t0 = tile * TILE;
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        if (lo == hi)
            continue;
        __syncthreads();
        stage_tile(a, tile, w);
        if (dd && ti.set != dd_set) {
            // block indices are relative to the set's own filter
            for (uint32_t q = threadIdx.x; q < FILL_DD; q += BLOCK)
                dd[q] = ~0ull;
            dd_set = ti.set;
        }
        __syncthreads();
        const TileSet ts = tile_set_of(a, pool, ti.set);
        uint32_t si = hi;
        uint64_t gs = 0, ge = 0;
        for (uint32_t it = 0; it < TILE / BLOCK; ++it) {
            const uint64_t p = t0 + it * BLOCK + threadIdx.x;
            if (p >= ge) {
                si = find_string(a.strings, lo, hi, p);
                gs = si != hi ? a.strings[si].gstart : ~0ull;
                ge = si != hi ? a.strings[si].gend : 0;
            }
            if (p < gs || p + L > ge)
                continue;
            const uint32_t r = (uint32_t)(p - t0) + 32;
            const Strands<T> e = strands(KT<T>::window(w, r, L), L);
            if (a.classes) {
                // a round inserts the edges next to a k-mer of its class
                T pre, suf;
                edge_kmers(e, a.k, single, &pre, &suf);
                if (!in_class(class_subrange(pre), ts.cls_lo, ts.cls_hi) &&
                    !in_class(class_subrange(suf), ts.cls_lo, ts.cls_hi))
                    continue;
            }
            my_atomics += BLOCKED ? insert_blocked(ts.f, e, a.k, single, dd)
                                  : insert_standard(ts.f, e, single);
        }
    }
    if (my_atomics)
        atomicAdd(&block_atomics, (unsigned long long)my_atomics);
    __syncthreads();
    if (threadIdx.x == 0 && block_atomics)
        atomicAdd(&cnt->fill_atomics, block_atomics);
}

static size_t fill_lds_bytes(const SeqArgs &a, bool blocked) {
    return blocked && a.fill_dedup ? FILL_DD * sizeof(unsigned long long) : 0;
}

hipError_t launch_fill(int W, const SeqArgs &a, const BloomArgs &pool, Counters *cnt,
                       uint32_t grid, hipStream_t s) {
    if (a.n_tiles == 0)
        return hipSuccess;
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        if (pool.blocked)
            hipLaunchKernelGGL((k_fill<T, true>), dim3(grid), dim3(BLOCK), fill_lds_bytes(a, true),
                               s, a, pool, cnt);
        else
            hipLaunchKernelGGL((k_fill<T, false>), dim3(grid), dim3(BLOCK), 0, s, a, pool, cnt);
        return hipGetLastError();
    });
}

// ------------------------------------------------------- binned fill (a1)
//
// The same filter as k_fill, built without random atomics: a chunk of tiles
// at a time, every edge's filter effect becomes an item, the items are
// partitioned by region of the pool in two streaming passes (bucket, then
// region within the bucket), and each region is applied in LDS.  A filter is
// the OR of its edges' bits, so the order of application does not matter.
//
//   k_bin_count    per workgroup (a static range of the chunk's tiles): its
//                  items, staged in position order, and counted per bucket
//   k_bin_scan     exclusive scan of the counts, bucket-major: each
//                  (bucket, workgroup) pair gets its own range of items_a
//   k_bin_scatter  the staged items, each written to its pair's range
//   k_bin_split    per bucket: its items counted and written by region, as
//                  4-byte items (the block's low bits and the bits it sets)
//
// The scatter and the split sort each batch by destination in LDS first, so
// that a destination's items of the batch leave as one contiguous run.
//   k_bin_apply    per region: the region's blocks in LDS, its items ORed in,
//                  the blocks written back

constexpr uint32_t BIN_BUCKET_SHIFT = 16 + BIN_REGION_LOG2 + BIN_SUB_LOG2;
constexpr uint32_t BIN_REGION_SHIFT = 16 + BIN_REGION_LOG2;
constexpr uint32_t BIN_PER = TILE / BLOCK;  // positions per thread per tile
static_assert(BIN_MAX_BUCKETS % BLOCK == 0, "bucket scan: whole counters per thread");

// The filter effect of edge e: its block in the pool (the set's first block
// plus its block in the set's filter), and the offset, stride and pair that
// fix its bits there.
template <class T>
__device__ __forceinline__ uint64_t bin_item(const BloomArgs &f, uint64_t block0,
                                             const Strands<T> &e, uint32_t k, bool single) {
    const T mid_ones = KT<T>::ones(2 * (k - 1));
    const uint32_t x = (uint32_t)(e.fwd >> (2 * k)), y = (uint32_t)(e.fwd & 3);
    const MiddleKey key = middle_key((T)((e.fwd >> 2) & mid_ones), (T)((e.rc >> 2) & mid_ones),
                                     single, f.mask >> 6);
    const uint32_t j = pair_index(key.orient, x, y, e.fwd <= e.rc);
    return (block0 + key.block) << 16 | (uint64_t)(key.a | key.d << 6 | j << 12);
}

// Every item of this workgroup's tiles (a contiguous share of the chunk), a
// tile at a time: per thread, v[q] is the item of position
// tile*TILE + q*BLOCK + thread, or BIN_NONE.  The edges are those k_fill
// inserts: every (k+1)-mer within a string, of the round's class when there
// are rounds.  tile_done(tile, v) is called by the whole workgroup for
// every tile of the share.
template <class T, class F>
__device__ __forceinline__ void bin_walk(const SeqArgs &a, const BloomArgs &pool,
                                         const BinArgs &b, uint64_t *w, F &&tile_done) {
    const uint32_t L = a.k + 1;
    const bool single = a.single != 0;
    const uint64_t n = b.tile_hi - b.tile_lo;
    const uint64_t per = (n + b.grid - 1) / b.grid;
    const uint64_t t_lo = b.tile_lo + min(n, (uint64_t)blockIdx.x * per);
    const uint64_t t_hi = b.tile_lo + min(n, (uint64_t)(blockIdx.x + 1) * per);
    for (uint64_t tile = t_lo; tile < t_hi; ++tile) {
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        uint64_t v[BIN_PER];
        if (lo == hi) {
#pragma unroll
            for (uint32_t q = 0; q < BIN_PER; ++q)
                v[q] = BIN_NONE;
            tile_done(tile, v);
            continue;
        }
        const uint64_t t0 = tile * TILE;
        __syncthreads();
        stage_tile(a, tile, w);
        __syncthreads();
        const TileSet ts = tile_set_of(a, pool, ti.set);
        const uint64_t block0 = a.sets[ti.set].bloom_off >> 1;
        uint32_t si = hi;
        uint64_t gs = 0, ge = 0;
#pragma unroll
        for (uint32_t q = 0; q < BIN_PER; ++q) {
            v[q] = BIN_NONE;
            const uint64_t p = t0 + q * BLOCK + threadIdx.x;
            if (p >= ge) {
                si = find_string(a.strings, lo, hi, p);
                gs = si != hi ? a.strings[si].gstart : ~0ull;
                ge = si != hi ? a.strings[si].gend : 0;
            }
            if (p < gs || p + L > ge)
                continue;
            const uint32_t r = (uint32_t)(p - t0) + 32;
            const Strands<T> e = strands(KT<T>::window(w, r, L), L);
            if (a.classes) {
                T pre, suf;
                edge_kmers(e, a.k, single, &pre, &suf);
                if (!in_class(class_subrange(pre), ts.cls_lo, ts.cls_hi) &&
                    !in_class(class_subrange(suf), ts.cls_lo, ts.cls_hi))
                    continue;
            }
            v[q] = bin_item(ts.f, block0, e, a.k, single);
        }
        tile_done(tile, v);
    }
}

// sorted_write by a field of the item: bin (v >> SHIFT) mod NB.
template <uint32_t NB, uint32_t NT, uint32_t PER, uint32_t SHIFT>
__device__ __forceinline__ void sorted_write(const uint64_t (&v)[PER], uint32_t *cnt,
                                             uint32_t *start, uint32_t *wtot, uint32_t *total,
                                             uint64_t *srt, uint64_t *cursor, uint64_t *out) {
    sorted_write_by<NB, NT, PER>(
        v, [](uint64_t x) { return (uint32_t)(x >> SHIFT) & (NB - 1); }, cnt, start, wtot, total,
        srt, cursor, out);
}

// The items of the chunk, one slot per position (BIN_NONE where there is
// none), written to items_b in position order; per workgroup, its items per
// bucket.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_bin_count(SeqArgs a, BloomArgs pool, BinArgs b) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint32_t hist[BIN_MAX_BUCKETS];
    for (uint32_t i = threadIdx.x; i < BIN_MAX_BUCKETS; i += BLOCK)
        hist[i] = 0;
    __syncthreads();
    uint64_t *stage = b.items_b;
    bin_walk<T>(a, pool, b, w, [&](uint64_t tile, const uint64_t (&v)[BIN_PER]) {
        uint64_t *dst = stage + (tile - b.tile_lo) * TILE + threadIdx.x;
#pragma unroll
        for (uint32_t q = 0; q < BIN_PER; ++q) {
            dst[q * BLOCK] = v[q];
            if (v[q] != BIN_NONE)
                atomicAdd(&hist[v[q] >> BIN_BUCKET_SHIFT], 1u);
        }
    });
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < b.n_buckets; i += BLOCK)
        b.counts[(uint64_t)i * b.grid + blockIdx.x] = hist[i];
}

// Each workgroup's staged items (the positions of its share of the chunk,
// as k_bin_count walked them) written to its (bucket, workgroup) ranges of
// items_a, a sorted batch of BIN_SCATTER_PER items per thread at a time.
__global__ __launch_bounds__(BIN_SCATTER_BLOCK) void k_bin_scatter(BinArgs b) {
    constexpr uint32_t NT = BIN_SCATTER_BLOCK, PER = BIN_SCATTER_PER;
    __shared__ uint64_t cursor[BIN_MAX_BUCKETS];
    __shared__ uint32_t cnt[BIN_MAX_BUCKETS];
    __shared__ uint32_t start[BIN_MAX_BUCKETS];
    __shared__ uint64_t srt[NT * PER];
    __shared__ uint32_t wtot[NT / 64];
    __shared__ uint32_t total;
    for (uint32_t i = threadIdx.x; i < BIN_MAX_BUCKETS; i += NT) {
        cursor[i] = i < b.n_buckets ? b.offsets[(uint64_t)i * b.grid + blockIdx.x] : 0;
        cnt[i] = 0;
    }
    __syncthreads();
    const uint64_t n = b.tile_hi - b.tile_lo;
    const uint64_t per = (n + b.grid - 1) / b.grid;
    const uint64_t p_lo = min(n, (uint64_t)blockIdx.x * per) * TILE;
    const uint64_t p_hi = min(n, (uint64_t)(blockIdx.x + 1) * per) * TILE;
    const uint64_t *stage = b.items_b;
    // every thread runs the same number of batches (the workgroup syncs in each)
    for (uint64_t i0 = p_lo; i0 < p_hi; i0 += PER * NT) {
        uint64_t v[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint64_t j = i0 + (uint64_t)q * NT + threadIdx.x;
            v[q] = j < p_hi ? stage[j] : BIN_NONE;
        }
        sorted_write<BIN_MAX_BUCKETS, NT, PER, BIN_BUCKET_SHIFT>(v, cnt, start, wtot, &total, srt,
                                                                cursor, b.items_a);
    }
}

__global__ __launch_bounds__(BIN_SCAN_BLOCK) void k_bin_scan(const uint32_t *counts, uint64_t n,
                                                            uint64_t *offsets) {
    bin_offsets_scan(counts, n, offsets);
}

// One workgroup per bucket: its items (the ranges of all its pairs, which
// lie back to back) counted by region, then written region by region into
// the same range of items_b, a sorted batch at a time; region_off gets each
// region's first item.
__global__ __launch_bounds__(BIN_SPLIT_BLOCK) void k_bin_split(BinArgs b) {
    constexpr uint32_t NT = BIN_SPLIT_BLOCK, PER = BIN_SPLIT_PER;
    __shared__ uint32_t cnt[BIN_SUB];
    __shared__ uint32_t start[BIN_SUB];
    __shared__ uint64_t cursor[BIN_SUB];
    __shared__ uint64_t srt[NT * PER];
    __shared__ uint32_t wtot[NT / 64];
    __shared__ uint32_t total;
    const uint32_t bk = blockIdx.x;
    const uint64_t lo = b.offsets[(uint64_t)bk * b.grid];
    const uint64_t hi = b.offsets[(uint64_t)(bk + 1) * b.grid];
    for (uint32_t i = threadIdx.x; i < BIN_SUB; i += NT)
        cnt[i] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += PER * NT) {
        uint64_t v[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint64_t j = i + (uint64_t)q * NT;
            v[q] = j < hi ? b.items_a[j] : BIN_NONE;
        }
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q)
            if (v[q] != BIN_NONE)
                atomicAdd(&cnt[(uint32_t)(v[q] >> BIN_REGION_SHIFT) & (BIN_SUB - 1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t c = lo;
        for (uint32_t q = 0; q < BIN_SUB; ++q) {
            cursor[q] = c;
            b.region_off[(uint64_t)bk * BIN_SUB + q] = c;
            c += cnt[q];
            cnt[q] = 0;
        }
        if (bk + 1 == b.n_buckets)
            b.region_off[(uint64_t)b.n_buckets * BIN_SUB] = c;
    }
    __syncthreads();
    // every thread runs the same number of batches (the workgroup syncs in each)
    for (uint64_t i0 = lo; i0 < hi; i0 += PER * NT) {
        uint64_t v[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint64_t j = i0 + (uint64_t)q * NT + threadIdx.x;
            v[q] = j < hi ? b.items_a[j] : BIN_NONE;
        }
        // out as 4-byte items: the block within its region and the bits it sets
        sorted_write_by<BIN_SUB, NT, PER>(
            v, [](uint64_t x) { return (uint32_t)(x >> BIN_REGION_SHIFT) & (BIN_SUB - 1); }, cnt,
            start, wtot, &total, srt, cursor, (uint32_t *)b.items_b);
    }
}

// One workgroup per region: the region's blocks (zero in the first chunk)
// in LDS, its items ORed in, the blocks written back.  Counts the items that
// set a bit not yet set.
__global__ __launch_bounds__(BIN_APPLY_BLOCK) void k_bin_apply(BloomArgs pool, BinArgs b,
                                                             Counters *cnt) {
    constexpr uint32_t NT = BIN_APPLY_BLOCK;
    __shared__ __align__(16) unsigned long long reg[BIN_REGION];
    __shared__ uint32_t fresh_wg;
    const uint64_t r = blockIdx.x;
    const uint64_t blk0 = r << BIN_REGION_LOG2;
    const uint32_t nb = (uint32_t)min((uint64_t)BIN_REGION, b.n_blocks - blk0);
    unsigned long long *blocks = (unsigned long long *)pool.words + blk0;
    if (threadIdx.x == 0)
        fresh_wg = 0;
    // blocks in pairs (the pool and every region start 16-byte aligned)
    const uint32_t np = nb / 2;
    ulonglong2 *reg2 = (ulonglong2 *)reg;
    const ulonglong2 *src2 = (const ulonglong2 *)blocks;
    for (uint32_t i = threadIdx.x; i < np; i += NT)
        reg2[i] = b.first ? make_ulonglong2(0, 0) : src2[i];
    if (threadIdx.x == 0 && (nb & 1))
        reg[nb - 1] = b.first ? 0ull : blocks[nb - 1];
    __syncthreads();
    const uint64_t lo = b.region_off[r], hi = b.region_off[r + 1];
    const uint32_t *items = (const uint32_t *)b.items_b;  // 4-byte items of the split
    constexpr uint32_t U = 4;
    uint32_t fresh = 0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += U * NT) {
        uint32_t v[U];
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            const uint64_t j = i + (uint64_t)q * NT;
            v[q] = j < hi ? items[j] : 0u;
        }
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            if (i + (uint64_t)q * NT < hi) {
                const uint32_t local = (v[q] >> 16) & (BIN_REGION - 1);
                const unsigned long long m = pair_mask(v[q] & 63, (v[q] >> 6) & 63,
                                                       (v[q] >> 12) & 15, pool.h);
                const unsigned long long old = atomicOr(&reg[local], m);
                fresh += (old & m) != m;
            }
        }
    }
    if (fresh)
        atomicAdd(&fresh_wg, fresh);
    __syncthreads();
    ulonglong2 *dst2 = (ulonglong2 *)blocks;
    for (uint32_t i = threadIdx.x; i < np; i += NT)
        dst2[i] = reg2[i];
    if (threadIdx.x == 0 && (nb & 1))
        blocks[nb - 1] = reg[nb - 1];
    if (threadIdx.x == 0 && fresh_wg)
        atomicAdd(&cnt->fill_atomics, (unsigned long long)fresh_wg);
}

hipError_t launch_fill_binned(int W, const SeqArgs &a, const BloomArgs &pool, Counters *cnt,
                              BinArgs b, uint32_t tiles_per_chunk, hipStream_t s) {
    if (a.n_tiles == 0)
        return hipSuccess;
    const uint64_t regions = (b.n_blocks + BIN_REGION - 1) >> BIN_REGION_LOG2;
    const uint64_t n_counts = (uint64_t)b.n_buckets * b.grid;
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        for (uint64_t t0 = 0; t0 < a.n_tiles; t0 += tiles_per_chunk) {
            b.tile_lo = t0;
            b.tile_hi = min(a.n_tiles, t0 + tiles_per_chunk);
            b.first = t0 == 0 ? 1u : 0u;
            hipLaunchKernelGGL(k_bin_count<T>, dim3(b.grid), dim3(BLOCK), 0, s, a, pool, b);
            hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(BIN_SCAN_BLOCK), 0, s, b.counts, n_counts,
                               b.offsets);
            hipLaunchKernelGGL(k_bin_scatter, dim3(b.grid), dim3(BIN_SCATTER_BLOCK), 0, s, b);
            hipLaunchKernelGGL(k_bin_split, dim3(b.n_buckets), dim3(BIN_SPLIT_BLOCK), 0, s, b);
            hipLaunchKernelGGL(k_bin_apply, dim3((uint32_t)regions), dim3(BIN_APPLY_BLOCK), 0, s,
                               pool, b, cnt);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    });
}

// --------------------------------------------------------------- query (a2)

// Standard layout: membership of the six neighbour (k+1)-mers, probed level
// by level.  True when some neighbour has all h bits set.
template <class T>
__device__ __forceinline__ bool any_present_standard(const BloomArgs &f, const Strands<T> &st,
                                                     uint32_t k, uint32_t pa, uint32_t sb,
                                                     bool single, uint32_t &probes) {
    uint64_t h1[6], h2[6];
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j) {
        // out-neighbour v.c for the j-th base c other than the successor
        const uint32_t c = j + (j >= sb);
        Strands<T> o;
        o.fwd = (st.fwd << 2) | (T)c;
        o.rc = st.rc | ((T)(3 - c) << (2 * k));
        const BloomHash bo = bloom_hash(norm(o, single));
        h1[j] = bo.h1;
        h2[j] = bo.h2;
        // in-neighbour d.v for the j-th base d other than the predecessor
        const uint32_t d = j + (j >= pa);
        Strands<T> n;
        n.fwd = ((T)d << (2 * k)) | st.fwd;
        n.rc = (st.rc << 2) | (T)(3 - d);
        const BloomHash bn = bloom_hash(norm(n, single));
        h1[3 + j] = bn.h1;
        h2[3 + j] = bn.h2;
    }
    uint32_t alive = 0x3F;
    for (uint32_t t = 0; t < f.h; ++t) {
        probes += __popc(alive);
        uint32_t v[6];
        uint32_t b[6];
#pragma unroll
        for (int n = 0; n < 6; ++n) {
            const uint64_t idx = (h1[n] + (uint64_t)t * h2[n]) & f.mask;
            b[n] = (uint32_t)(idx & 31);
            v[n] = ((alive >> n) & 1u) ? __hip_atomic_load(&f.words[idx >> 5], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                        : 0u;
        }
#pragma unroll
        for (int n = 0; n < 6; ++n)
            if (!((v[n] >> b[n]) & 1u))
                alive &= ~(1u << n);
        if (!alive)
            return false;
    }
    return true;
}

// Pair tests in rotation form.  Pair j's bits (a + (j*h + t)*d) mod 64,
// t < h, are the key's template sum_t 2^(t*d mod 64) rotated left by
// s = a + j*hd, hd = h*d mod 64; the template depends on the odd stride d
// only, so a workgroup keeps the 32 of them in LDS.  In the query, the pair
// index of the edge through base c is affine in c for a non-palindromic
// middle: s = base + c*step (mod 64).
struct PairKey {
    uint32_t a, d, hd, orient;
};

__device__ __forceinline__ uint32_t pack_key(const MiddleKey &m, uint32_t h) {
    return m.a | m.d << 6 | ((h * m.d) & 63u) << 12 | m.orient << 18;
}

__device__ __forceinline__ PairKey unpack_key(uint32_t x) {
    return PairKey{x & 63u, (x >> 6) & 63u, (x >> 12) & 63u, x >> 18};
}

// All bits of template t, rotated left by s (mod 64), set in w.
__device__ __forceinline__ bool rot_all(uint64_t w, uint64_t t, uint32_t s) {
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    const bool sw = (s & 32u) != 0;  // rotating by 32 swaps the halves
    const uint32_t x = sw ? lo : hi, y = sw ? hi : lo;
    const uint32_t rlo = __builtin_amdgcn_alignbit(x, y, s);
    const uint32_t rhi = __builtin_amdgcn_alignbit(y, x, s);
    return ((~rlo & (uint32_t)t) | (~rhi & (uint32_t)(t >> 32))) == 0;
}

// Value of the lane below (DPP wave shift right by one); lane 0 gets lane0.
__device__ __forceinline__ uint32_t from_below(uint32_t x, uint32_t lane0) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)lane0, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t from_below(uint64_t x, uint64_t lane0) {
    return ((uint64_t)from_below((uint32_t)(x >> 32), (uint32_t)(lane0 >> 32)) << 32) |
           from_below((uint32_t)x, (uint32_t)lane0);
}

__device__ __forceinline__ uint64_t lane63(uint64_t x) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), 63) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 63);
}

// Blocked layout: the three out-edges against the out-middle block wo, the
// three in-edges against the in-middle block wi.  Only a palindromic middle
// (orientation 2) needs the edge's own orientation, per edge.
template <class T>
__device__ __forceinline__ bool any_present_blocked(const Strands<T> &st, uint32_t k, uint32_t pa,
                                                    uint32_t sb, const PairKey &ko, uint64_t to,
                                                    uint64_t wo, const PairKey &ki, uint64_t ti,
                                                    uint64_t wi) {
    const uint32_t v0 = (uint32_t)(st.fwd >> (2 * (k - 1)));
    const uint32_t vk = (uint32_t)(st.fwd & 3);
    // out-edge v.c has pair 4*v0 + c, or 15 - 4c - v0 read reversed; in-edge
    // d.v has pair 4d + vk, or 15 - 4*vk - d reversed
    const bool fo = ko.orient == 1, fi = ki.orient == 1;
    uint32_t so[3], si[3];
    {
        const uint32_t bo = ko.a + __umul24(fo ? 15 - v0 : 4 * v0, ko.hd);
        const uint32_t po = fo ? 64 - 4 * ko.hd : ko.hd;
        const uint32_t bi = ki.a + __umul24(fi ? 15 - 4 * vk : vk, ki.hd);
        const uint32_t pi = fi ? 64 - ki.hd : 4 * ki.hd;
#pragma unroll
        for (uint32_t j = 0; j < 3; ++j) {
            so[j] = bo + __umul24(j + (j >= sb), po);
            si[j] = bi + __umul24(j + (j >= pa), pi);
        }
    }
    const bool pal = ko.orient == 2 || ki.orient == 2;
    if (__builtin_amdgcn_ballot_w64(pal)) {
        if (pal) {
#pragma unroll
            for (uint32_t j = 0; j < 3; ++j) {
                if (ko.orient == 2) {
                    const uint32_t c = j + (j >= sb);
                    const T of = (st.fwd << 2) | (T)c;
                    const T orc = st.rc | ((T)(3 - c) << (2 * k));
                    so[j] = ko.a + ko.hd * pair_index(2, v0, c, of <= orc);
                }
                if (ki.orient == 2) {
                    const uint32_t d = j + (j >= pa);
                    const T inf = ((T)d << (2 * k)) | st.fwd;
                    const T inr = (st.rc << 2) | (T)(3 - d);
                    si[j] = ki.a + ki.hd * pair_index(2, d, vk, inf <= inr);
                }
            }
        }
    }
    bool present = false;
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j)
        present |= rot_all(wo, to, so[j]) | rot_all(wi, ti, si[j]);
    return present;
}

template <class T, bool BLOCKED, bool CLASSES>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(KT<T>::W == 1 ? 5 : 1)))
void k_query(SeqArgs a, BloomArgs pool, SentArgs sa,
                                                 uint64_t *c1, uint64_t *c1u, uint32_t round,
                                                 Counters *cnt, uint32_t *hll_out) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint32_t pf[(1u << PF_MAX_LOG2) / 32];
    __shared__ uint32_t hll[HLL_M];
    __shared__ uint64_t tmpl[32];  // pair template of odd stride d at d >> 1
    __shared__ unsigned long long block_probes, cand_lds;
    SetSum cand = setsum_begin();
    const uint32_t k = a.k;
    const bool single = a.single != 0;
    const T *sent = (const T *)sa.table;
    const uint32_t lane = threadIdx.x & 63;
    const T mid_ones = KT<T>::ones(2 * (k - 1));
    for (uint32_t i = threadIdx.x; i < (1u << sa.pf_log2) / 32; i += BLOCK)
        pf[i] = sa.prefilter[i];
    for (uint32_t i = threadIdx.x; i < HLL_M; i += BLOCK)
        hll[i] = 0;
    if (BLOCKED && threadIdx.x < 32) {
        const uint32_t d = 2 * threadIdx.x + 1;
        uint64_t m = 0;
        for (uint32_t t = 0; t < pool.h; ++t)
            m |= 1ull << ((t * d) & 63u);
        tmpl[threadIdx.x] = m;
    }
    if (threadIdx.x == 0)
        block_probes = 0;
    uint32_t my_probes = 0;

    RunCursor rc = run_cursor(a, a.chunk);
    for (uint64_t tile; run_next(a, rc, &tile);) {
        const uint64_t t0 = tile * TILE;
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        if (lo == hi) {
            // no string touches this tile: all-zero candidate words
            if (threadIdx.x < TILE / 64) {
                c1[tile * (TILE / 64) + threadIdx.x] = 0;
                if (c1u && round == 0)
                    c1u[tile * (TILE / 64) + threadIdx.x] = 0;
            }
            continue;
        }
        __syncthreads();
        stage_tile(a, tile, w);
        __syncthreads();
        const TileSet ts = tile_set_of(a, pool, ti.set);
        const unsigned long long *blocks = (const unsigned long long *)ts.f.words;
        setsum_switch(cand, ts.set, &cand_lds, &a.set_cnt[0].candidates, SETCNT_STRIDE);
        uint32_t si = hi;
        uint64_t gs = 0, ge = 0;
        // each wave walks its own run of consecutive positions, 64 at a time;
        // lane 63's out-middle key and block carry to the next step's lane 0
        const uint64_t run0 = t0 + (uint64_t)(threadIdx.x >> 6) * (TILE / (BLOCK / 64));
        uint32_t carry_key = 0;
        uint64_t carry_w = 0, carry_g = 0;
        for (uint32_t it = 0; it < TILE / BLOCK; ++it) {
            const uint64_t p = run0 + it * 64 + lane;
            if (p >= ge) {
                si = find_string(a.strings, lo, hi, p);
                gs = si != hi ? a.strings[si].gstart : ~0ull;
                ge = si != hi ? a.strings[si].gend : 0;
            }
            const bool valid = p >= gs && p + k <= ge;
            const uint32_t r = (uint32_t)(p - t0) + 32;
            Strands<T> st;
            st.fwd = 0;
            st.rc = 0;
            if (valid)
                st = strands(KT<T>::window(w, r, k), k);
            // evaluated in this round: every valid position, or with classes
            // those whose k-mer is in the round's class
            bool live = valid;
            if (CLASSES && valid)
                live = in_class(class_subrange(norm(st, single)), ts.cls_lo, ts.cls_hi);
            uint32_t kout = 0, kin = 0;
            unsigned long long wo = 0, wi = 0;
            uint64_t gout = 0, gin = 0;  // G of the out- and in-middle
            if (BLOCKED) {
                // a valid lane takes its out-middle key and block when it or
                // the position above is evaluated; the position above uses
                // them as its in-middle (an evaluated position that is not a
                // string start has a valid predecessor in its string).  Lane
                // 63's position above is the next step's lane 0.
                const bool live_above = CLASSES ? __shfl_down(live, 1, 64) != 0 : true;
                const bool need = !CLASSES || live || lane == 63 || live_above;
                if (valid && need) {
                    const MiddleKey m = middle_key((T)(st.fwd & mid_ones), (T)(st.rc >> 2), single,
                                                   ts.f.mask >> 6);
                    kout = pack_key(m, ts.f.h);
                    gout = m.g;
                    wo = __hip_atomic_load(&blocks[m.block], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    ++my_probes;
                }
                kin = from_below(kout, carry_key);
                wi = from_below((uint64_t)wo, carry_w);
                gin = from_below(gout, carry_g);
                carry_key = (uint32_t)__builtin_amdgcn_readlane((int)kout, 63);
                carry_w = lane63(wo);
                carry_g = lane63(gout);
                if (it == 0 && lane == 0 && live && p > gs) {
                    // the position before is in another wave's run
                    const MiddleKey m = middle_key((T)(st.fwd >> 2), (T)(st.rc & mid_ones), single,
                                                   ts.f.mask >> 6);
                    kin = pack_key(m, ts.f.h);
                    gin = m.g;
                    wi = __hip_atomic_load(&blocks[m.block], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    ++my_probes;
                }
            }
            bool mark = false;
            T canon = 0;
            if (live) {
                canon = norm(st, single);
                if (p == gs || p + k == ge) {
                    mark = true;  // first or last k-mer of its string
                } else if (BLOCKED) {
                    // the neighbour test needs only the blocks already loaded,
                    // so it goes first: a marked position skips the sentinel
                    // lookup (a probe of the sentinel table on a prefilter hit)
                    const uint32_t pa = base_at(w, r - 1), sb = base_at(w, r + k);
                    const PairKey ko = unpack_key(kout), ki = unpack_key(kin);
                    mark = any_present_blocked(st, k, pa, sb, ko, tmpl[ko.d >> 1], wo, ki,
                                               tmpl[ki.d >> 1], wi) ||
                           is_sentinel(canon, pf, sa.pf_log2, sent + ts.sent_off, ts.sent_log2);
                } else if (is_sentinel(canon, pf, sa.pf_log2, sent + ts.sent_off, ts.sent_log2)) {
                    mark = true;
                } else {
                    const uint32_t pa = base_at(w, r - 1), sb = base_at(w, r + k);
                    mark = any_present_standard(ts.f, st, k, pa, sb, single, my_probes);
                }
            }
            const uint64_t word = ballot64(mark);
            if (lane == 0) {
                c1[p >> 6] = word;
                if (c1u)
                    c1u[p >> 6] = round ? c1u[p >> 6] | word : word;
                cand.v += (unsigned long long)__popcll(word);
            }
            if (a.sketch && mark) {
                // item hash of the candidate k-mer: with the blocked filter the sum
                // of its two middles' G values (an unordered pair, the same for
                // both orientations; a string's first k-mer hashes its first
                // middle here), else its table hash
                uint64_t hv;
                if (BLOCKED) {
                    if (p == gs)
                        gin = middle_key((T)(st.fwd >> 2), (T)(st.rc & mid_ones), single, 0).g;
                    hv = gin + gout;
                } else {
                    hv = slot_hash(canon);
                }
                const uint32_t reg = (uint32_t)(hv >> (64 - HLL_LOG2));
                const uint64_t rest = hv << HLL_LOG2;
                const uint32_t rank = rest ? (uint32_t)__clzll(rest) + 1 : 64 - HLL_LOG2 + 1;
                atomicMax(&hll[reg], rank);
            }
        }
    }
    setsum_flush(cand, &cand_lds, &a.set_cnt[0].candidates, SETCNT_STRIDE);
    if (my_probes)
        atomicAdd(&block_probes, (unsigned long long)my_probes);
    __syncthreads();
    if (threadIdx.x == 0 && block_probes)
        atomicAdd(&cnt->query_probes, block_probes);
    if (a.sketch) {
        for (uint32_t i = threadIdx.x; i < HLL_M; i += BLOCK) {
            const uint32_t v = hll[i];
            if (v && v > __hip_atomic_load(&hll_out[i], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(&hll_out[i], v);
        }
    }
}

template <class T, bool BLOCKED>
static void query_t(const SeqArgs &a, const BloomArgs &pool, const SentArgs &sa, uint64_t *c1,
                    uint64_t *c1u, uint32_t round, Counters *cnt, uint32_t *hll, uint32_t grid,
                    hipStream_t s) {
    if (a.classes)
        hipLaunchKernelGGL((k_query<T, BLOCKED, true>), dim3(grid), dim3(BLOCK), 0, s, a, pool,
                           sa, c1, c1u, round, cnt, hll);
    else
        hipLaunchKernelGGL((k_query<T, BLOCKED, false>), dim3(grid), dim3(BLOCK), 0, s, a, pool,
                           sa, c1, c1u, round, cnt, hll);
}

hipError_t launch_query(int W, const SeqArgs &a, const BloomArgs &pool, const SentArgs &sa,
                        uint64_t *c1, uint64_t *c1u, uint32_t round, Counters *cnt,
                        uint32_t *hll, uint32_t grid, hipStream_t s) {
    if (a.n_tiles == 0)
        return hipSuccess;
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        if (pool.blocked)
            query_t<T, true>(a, pool, sa, c1, c1u, round, cnt, hll, grid, s);
        else
            query_t<T, false>(a, pool, sa, c1, c1u, round, cnt, hll, grid, s);
        return hipGetLastError();
    });
}

// ------------------------------------------------- class census (rounds)

// Per set, CLASS_Q counters: every (k+1)-mer adds one to the subrange of
// each distinct class subrange among its two normalised k-mers (Multiple
// Rounds section: counters estimate the (k+1)-mers that touch each class).
// A workgroup counts in LDS and adds its counts to the set's counters when
// its tiles move to another set, and at the end.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_census(SeqArgs a, unsigned long long *counters) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint32_t hist[CLASS_Q];
    const uint32_t L = a.k + 1;
    const bool single = a.single != 0;
    for (uint32_t i = threadIdx.x; i < CLASS_Q; i += BLOCK)
        hist[i] = 0;
    uint32_t cur_set = ~0u;
    auto flush = [&]() {
        __syncthreads();
        if (cur_set != ~0u)
            for (uint32_t i = threadIdx.x; i < CLASS_Q; i += BLOCK) {
                const uint32_t v = hist[i];
                if (v)
                    atomicAdd(&counters[(uint64_t)cur_set * CLASS_Q + i], (unsigned long long)v);
                hist[i] = 0;
            }
        __syncthreads();
    };
    RunCursor rc = run_cursor(a, a.chunk);
    for (uint64_t tile; run_next(a, rc, &tile);) {
        const uint64_t t0 = tile * TILE;
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        if (lo == hi)
            continue;
        if (ti.set != cur_set) {
            flush();
            cur_set = ti.set;
        }
        __syncthreads();
        stage_tile(a, tile, w);
        __syncthreads();
        uint32_t si = hi;
        uint64_t gs = 0, ge = 0;
        for (uint32_t it = 0; it < TILE / BLOCK; ++it) {
            const uint64_t p = t0 + it * BLOCK + threadIdx.x;
            if (p >= ge) {
                si = find_string(a.strings, lo, hi, p);
                gs = si != hi ? a.strings[si].gstart : ~0ull;
                ge = si != hi ? a.strings[si].gend : 0;
            }
            if (p < gs || p + L > ge)
                continue;
            const uint32_t r = (uint32_t)(p - t0) + 32;
            const Strands<T> e = strands(KT<T>::window(w, r, L), L);
            T pre, suf;
            edge_kmers(e, a.k, single, &pre, &suf);
            const uint32_t x = class_subrange(pre), y = class_subrange(suf);
            atomicAdd(&hist[x], 1u);
            if (y != x)
                atomicAdd(&hist[y], 1u);
        }
    }
    flush();
}

hipError_t launch_census(int W, const SeqArgs &a, unsigned long long *counters, uint32_t grid,
                         hipStream_t s) {
    hipError_t e = launch_zero(counters, (uint64_t)a.n_sets * CLASS_Q * 8, s);
    if (e != hipSuccess || a.n_tiles == 0)
        return e;
    return by_width(W, [&](auto tag) {
        hipLaunchKernelGGL(k_census<decltype(tag)>, dim3(grid), dim3(BLOCK), 0, s, a, counters);
        return hipGetLastError();
    });
}

// Greedy partition of the Multiple Rounds section on the device, one thread
// per set (the host's class_partition, for runs without host waits): class c
// takes the longest run of consecutive subranges, at least one while any
// remain, whose counter sum times the number of classes stays within the
// total; the last class takes every remaining subrange.
__global__ void k_partition(const unsigned long long *census, uint32_t n_sets, uint32_t rounds,
                            uint32_t *bounds) {
    const uint32_t set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets)
        return;
    const unsigned long long *e = census + (uint64_t)set * CLASS_Q;
    uint32_t *bound = bounds + (uint64_t)set * (rounds + 1);
    unsigned __int128 total = 0;
    for (uint32_t i = 0; i < CLASS_Q; ++i)
        total += e[i];
    uint32_t next = 0;
    for (uint32_t c = 0; c < rounds; ++c) {
        bound[c] = next;
        if (c + 1 == rounds) {
            next = CLASS_Q;
            continue;
        }
        unsigned __int128 sum = 0;
        for (uint32_t taken = 0; next < CLASS_Q; ++taken, ++next) {
            if (taken > 0 && (sum + e[next]) * rounds > total)
                break;
            sum += e[next];
        }
    }
    bound[rounds] = CLASS_Q;
}

__global__ void k_set_round(SetDesc *sets, const uint32_t *bounds, uint32_t n_sets,
                            uint32_t rounds, uint32_t round) {
    const uint32_t set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets)
        return;
    sets[set].cls_lo = bounds[(uint64_t)set * (rounds + 1) + round];
    sets[set].cls_hi = bounds[(uint64_t)set * (rounds + 1) + round + 1];
}

hipError_t launch_partition(const unsigned long long *census, uint32_t n_sets, uint32_t rounds,
                            uint32_t *bounds, hipStream_t s) {
    if (n_sets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_partition, dim3((n_sets + 63) / 64), dim3(64), 0, s, census, n_sets,
                       rounds, bounds);
    return hipGetLastError();
}

hipError_t launch_set_round(SetDesc *sets, const uint32_t *bounds, uint32_t n_sets,
                            uint32_t rounds, uint32_t round, hipStream_t s) {
    if (n_sets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_set_round, dim3((n_sets + 63) / 64), dim3(64), 0, s, sets, bounds,
                       n_sets, rounds, round);
    return hipGetLastError();
}

hipError_t pass1_occupancy(KernelId which, int W, bool blocked, bool fill_dedup, int *blocks) {
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        const void *fn = which == K_FILL
                             ? (blocked ? (const void *)k_fill<T, true> : (const void *)k_fill<T, false>)
                             : (blocked ? (const void *)k_query<T, true, false>
                                        : (const void *)k_query<T, false, false>);
        const size_t dyn = which == K_FILL && blocked && fill_dedup
                               ? FILL_DD * sizeof(unsigned long long) : 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, BLOCK, dyn);
    });
}

// ----------------------------------------------------- filter popcount per set

// Workgroup b counts words [b*chunk, (b+1)*chunk) of the pool; a thread adds
// its running count to a set's counter whenever its words cross into
// another set (set regions are consecutive in the pool).  At the end the
// threads whose last set is the last set of the chunk add in LDS first, so a
// chunk inside one set costs one device atomic.
__global__ __launch_bounds__(BLOCK) void k_popcount(const uint32_t *pool, uint64_t n,
                                                    uint64_t chunk, const uint64_t *starts,
                                                    uint32_t n_sets, SetCounters *sc) {
    __shared__ unsigned long long sum;
    __shared__ uint32_t last_set;
    const uint64_t b0 = blockIdx.x * chunk;
    const uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    uint32_t set = 0;
    unsigned long long c = 0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += BLOCK) {
        if (i < starts[set] || i >= starts[set + 1]) {
            if (c)
                atomicAdd(&sc[set].bloom_popcount, c);
            c = 0;
            uint32_t lo = 0, hi = n_sets;  // last set with starts[set] <= i
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (starts[mid] <= i)
                    lo = mid;
                else
                    hi = mid;
            }
            set = lo;
        }
        c += (unsigned long long)__popc(pool[i]);
    }
    if (threadIdx.x == 0) {
        sum = 0;
        // set of the chunk's last word
        uint32_t lo = 0, hi = n_sets;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (b1 > b0 && starts[mid] <= b1 - 1)
                lo = mid;
            else
                hi = mid;
        }
        last_set = lo;
    }
    __syncthreads();
    if (c) {
        if (set == last_set)
            atomicAdd(&sum, c);
        else
            atomicAdd(&sc[set].bloom_popcount, c);
    }
    __syncthreads();
    if (threadIdx.x == 0 && sum)
        atomicAdd(&sc[last_set].bloom_popcount, sum);
}

hipError_t launch_popcount(const uint32_t *pool, uint64_t n_words, const uint64_t *bloom_starts,
                           uint32_t n_sets, SetCounters *set_cnt, hipStream_t s) {
    if (n_words == 0 || n_sets == 0)
        return hipSuccess;
    const uint32_t grid = grid_for(n_words, 2048);
    const uint64_t chunk = (n_words + grid - 1) / grid;
    hipLaunchKernelGGL(k_popcount, dim3(grid), dim3(BLOCK), 0, s, pool, n_words, chunk,
                       bloom_starts, n_sets, set_cnt);
    return hipGetLastError();
}

}  // namespace tp
