// Second pass of Algorithm 2 (Filter-Junctions with E = exact set) over the
// first-pass candidates C1, for gfx950.
//
// The exact set is kept per vertex rather than per edge: an open-addressing
// table keyed by the normalised candidate k-mer v holds an 8-bit mask, bits
// 0-3 the bases c with c.v an edge (in) and bits 4-7 the bases c with v.c an
// edge (out), both for v in normalised orientation.  Every occurrence of an
// edge next to a candidate vertex lies next to a candidate position, because
// a candidate set never splits the positions of one normalised k-mer
// (Single Round section), so recording the predecessor and successor edge of
// every candidate position yields exactly the in/out edge sets that loop 2 of
// Algorithm 1 counts.  This stores one entry per distinct candidate k-mer
// instead of up to 8 per junction (Theoretical Analysis section).
//
//   k_record   loop 1: insert-or-find the normalised k-mer (atomicCAS on the
//              key word), then atomicOr its edge bits (load first, skip when
//              already set).  Two-word keys (k >= 32) claim the high word
//              with a pending bit, publish the low word, then release.
//   k_decide   loop 2: a candidate stays a junction when its k-mer is a
//              sentinel or has more than one in- or out-edge; one wave
//              ballot per 64 positions writes the J bitmap.
#include "device.hpp"

namespace tp {

// Stage a tile's packed words (as the first pass does) and its TILE / 64
// candidate-bitmap words in LDS, with one round of loads.
__device__ __forceinline__ void stage_tile2(const SeqArgs &a, uint64_t tile, uint64_t *w,
                                            const uint64_t *c1, uint64_t *cw) {
    int64_t w0 = (int64_t)(tile * TILE_WORDS) - 1;
    for (uint32_t i = threadIdx.x; i < STAGE_WORDS; i += blockDim.x) {
        int64_t gw = w0 + (int64_t)i;
        w[i] = (gw >= 0 && (uint64_t)gw < a.seq_words) ? a.seq[gw] : 0ull;
    }
    if (threadIdx.x >= BLOCK - TILE / 64)
        cw[threadIdx.x - (BLOCK - TILE / 64)] = c1[tile * (TILE / 64) + threadIdx.x -
                                                   (BLOCK - TILE / 64)];
}

__global__ void k_table_clear(unsigned long long *keys, unsigned long long *keys_hi,
                              uint32_t *masks, uint64_t cap) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < cap;
         i += (uint64_t)gridDim.x * blockDim.x) {
        keys[i] = EMPTY_KEY;
        if (keys_hi)
            keys_hi[i] = EMPTY_KEY;
        if (masks && (i & 3) == 0)
            masks[i >> 2] = 0;
    }
}

hipError_t launch_table_clear(int W, const TableArgs &pool, uint64_t slots, hipStream_t s) {
    if (slots == 0)
        return hipSuccess;
    uint64_t g = (slots + BLOCK - 1) / BLOCK;
    if (g > 16384)
        g = 16384;
    hipLaunchKernelGGL(k_table_clear, dim3((uint32_t)g), dim3(BLOCK), 0, s, pool.keys,
                       W >= 2 ? pool.keys_hi : nullptr, pool.packed ? nullptr : pool.masks, slots);
    return hipGetLastError();
}

// The table of a tile's set: the pools shifted to its region.
__device__ __forceinline__ TableArgs table_of(const SeqArgs &a, const TableArgs &pool,
                                              uint32_t set) {
    const SetDesc &d = a.sets[set];
    TableArgs t = pool;
    t.keys = pool.keys + d.table_off;
    if (pool.keys_hi)
        t.keys_hi = pool.keys_hi + d.table_off;
    if (pool.keys_mid)
        t.keys_mid = pool.keys_mid + 2 * d.table_off;
    if (pool.masks)
        t.masks = pool.masks + d.table_off / 4;
    t.cap_m = d.table_m;
    t.cap_e = d.table_e;
    t.lomask = (1ull << d.table_e) - 1;
    return t;
}

__device__ __forceinline__ unsigned long long ld(unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_mask(const uint32_t *masks, uint64_t s) {
    return __hip_atomic_load(&masks[s >> 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// OR edge bits m into slot s's mask byte, given an earlier reading mw of its
// word.  Mask bits are only ever set, so a stale reading costs at most an
// atomic that was not needed; it never skips one that was.
__device__ __forceinline__ void or_mask(uint32_t *masks, uint64_t s, uint32_t m, uint32_t mw) {
    const uint32_t mm = m << (8 * (uint32_t)(s & 3));
    if ((mw & mm) != mm)
        __hip_atomic_fetch_or(&masks[s >> 2], mm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int mask_byte(uint32_t mw, uint64_t s) {
    return (int)((mw >> (8 * (uint32_t)(s & 3))) & 0xFFu);
}

// A lookup starts at the key's home slot (first_slot) with that slot's word
// (first_word) and continues from there (*_from) to the next slots.  Two
// table modes, fixed per run (the kernels are instantiated for each):
//   P2    capacity 2^e: the home slot is the low e hash bits and probes wrap
//         at the capacity (a mask on the path from key to address);
//   any   capacity m << e (m < 2^32): m blocks of 2^e slots.  The home
//         slot's block is the high word of m * (top 32 hash bits), its slot
//         in the block the low e hash bits, uniform over [0, m << e); probes
//         wrap within the block, so a lookup never leaves its home block
//         (which lets the record insert block by block, see k_rbin_apply).
//
// Home slots are even, so a lookup can read the pair of slots it starts in
// with one 16-byte load (capacities and set regions are multiples of 64
// slots, so pairs never straddle them).
template <bool P2, class T>
__device__ __forceinline__ uint64_t first_slot(const TableArgs &t, T key) {
    const uint64_t h = slot_hash(key);
    if (P2)
        return h & t.lomask & ~1ull;
    const uint64_t top = __umulhi((uint32_t)(h >> 32), t.cap_m);
    return ((top << t.cap_e) | (h & t.lomask)) & ~1ull;
}

template <bool P2>
__device__ __forceinline__ uint64_t next_slot(const TableArgs &t, uint64_t s) {
    return P2 ? (s + 1) & t.lomask : (s & ~t.lomask) | ((s + 1) & t.lomask);
}

// The next pair of slots after the pair starting at s (s even).
template <bool P2>
__device__ __forceinline__ uint64_t next_pair(const TableArgs &t, uint64_t s) {
    return P2 ? (s + 2) & t.lomask : (s & ~t.lomask) | ((s + 2) & t.lomask);
}

typedef HIP_vector_type<unsigned long long, 2> u64x2;

// Words of slots s and s + 1 (s even), one 16-byte load.  The record reads
// pairs too, with plain loads: a word read stale can only be empty where a
// key now is (slots go from empty to a key, never back; mask bits are only
// set), which costs a failed claim or an extra OR, never a wrong answer.
__device__ __forceinline__ u64x2 load_pair(const TableArgs &t, uint64_t s) {
    return *(const u64x2 *)(t.keys + s);
}

// Insert-or-find of a one-word key by slot pairs, starting with the pair pr
// of slots s, s + 1 (s even): claim an empty slot by atomicCAS (packed slots
// take the key and its edge bits at once), or OR the edge bits into the
// key's slot.  1 when this call claimed a new slot, 0 when the key was
// present, -1 on overflow.
template <bool P2>
__device__ __forceinline__ int insert_pair(const TableArgs &t, uint64_t key, uint32_t m,
                                           uint64_t s, u64x2 pr, uint32_t &probes) {
    for (uint32_t i = 0; i < MAX_PROBE / 2; ++i) {
        if (i)
            pr = load_pair(t, s);
        ++probes;
#pragma unroll
        for (uint32_t half = 0; half < 2; ++half) {
            const uint64_t slot = s + half;
            unsigned long long cur = half ? pr.y : pr.x;
            if (t.packed) {
                if (cur == EMPTY_KEY) {
                    cur = atomicCAS(&t.keys[slot], EMPTY_KEY, (unsigned long long)((key << 8) | m));
                    if (cur == EMPTY_KEY)
                        return 1;
                }
                if ((cur >> 8) == key) {
                    if ((cur & m) != m)
                        __hip_atomic_fetch_or(&t.keys[slot], (unsigned long long)m,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    return 0;
                }
            } else {
                const uint32_t mw = ld_mask(t.masks, slot);
                int claimed = 0;
                if (cur == EMPTY_KEY) {
                    cur = atomicCAS(&t.keys[slot], EMPTY_KEY, (unsigned long long)key);
                    if (cur == EMPTY_KEY) {
                        cur = key;
                        claimed = 1;
                    }
                }
                if (cur == key) {
                    or_mask(t.masks, slot, m, mw);
                    return claimed;
                }
            }
        }
        s = next_pair<P2>(t, s);
    }
    return -1;
}

// Record reads slots other waves are writing (device-coherent loads); the
// decision reads a finished table (plain, cacheable loads).
__device__ __forceinline__ unsigned long long first_word(const TableArgs &t, uint64_t s, bool wide) {
    return wide ? ld(&t.keys_hi[s]) : ld(&t.keys[s]);
}

__device__ __forceinline__ unsigned long long first_word_ro(const TableArgs &t, uint64_t s,
                                                            bool wide) {
    return wide ? t.keys_hi[s] : t.keys[s];
}

// Insert-or-find of a one-word key, then OR of its edge bits, starting at
// slot s whose word is cur.  Packed slots hold key << 8 | mask (the key field
// of an empty slot, all ones, never equals a key of 2k <= 54 bits); split
// slots hold the key with the mask in a separate byte.  Returns 1 when this
// call claimed a new slot, 0 when the key was present, -1 on overflow.
template <bool P2>
__device__ __forceinline__ int insert_from(const TableArgs &t, uint64_t key, uint32_t m,
                                           uint64_t s, unsigned long long cur,
                                           uint32_t &probes) {
    for (uint32_t i = 0; i < MAX_PROBE; ++i) {
        ++probes;
        if (i)
            cur = ld(&t.keys[s]);
        const uint32_t mw = t.packed ? 0u : ld_mask(t.masks, s);  // issued with the key word
        if (t.packed) {
            if (cur == EMPTY_KEY) {
                cur = atomicCAS(&t.keys[s], EMPTY_KEY, (unsigned long long)((key << 8) | m));
                if (cur == EMPTY_KEY)
                    return 1;
            }
            if ((cur >> 8) == key) {
                if ((cur & m) != m)
                    __hip_atomic_fetch_or(&t.keys[s], (unsigned long long)m, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                return 0;
            }
        } else {
            int claimed = 0;
            if (cur == EMPTY_KEY) {
                cur = atomicCAS(&t.keys[s], EMPTY_KEY, (unsigned long long)key);
                if (cur == EMPTY_KEY) {
                    cur = key;
                    claimed = 1;
                }
            }
            if (cur == key) {
                or_mask(t.masks, s, m, mw);
                return claimed;
            }
        }
        s = next_slot<P2>(t, s);
    }
    return -1;
}

// Two-word keys: the high word (< 2^62 for k <= 63) is claimed with
// PENDING_BIT set, the low word written, then the high word published without
// the bit.  A finder that sees its high word pending reads the same slot
// again on the next trip.  The loop leaves only by a wave-wide vote, so no
// lane's claim-and-publish sits on a divergent exit path (which the
// structurised control flow would run after the loop, behind its own
// waiters): a claimer publishes in the same trip in which it claims.  The
// trip bound turns any unexpected livelock into an overflow report.
//
// Ordering without acquire/release: on a part whose dies have separate L2s,
// agent-scope acquire and release each cost a whole-L2 invalidate or
// write-back.  Every access here is instead a relaxed device-coherent atomic,
// performed at the coherence point.  The claimer writes the low word with an
// exchange and waits for its result before it issues the publishing
// exchange, so the low word is in place before any lane can see the high
// word published; a finder reads the low word only after its load of the
// published high word has returned.
// Multi-word keys: the top word lives in keys_hi, the others in keys (word
// 0) and keys_mid (words 1 and 2 of four-word keys).
__device__ __forceinline__ uint64_t top_word(u128 k) { return (uint64_t)(k >> 64); }
__device__ __forceinline__ uint64_t top_word(const u256 &k) { return k.w3; }

__device__ __forceinline__ unsigned long long xchg(unsigned long long *p, uint64_t v) {
    return __hip_atomic_exchange(p, (unsigned long long)v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
}

// Write the lower words of key into slot s; the result depends on every
// exchange's returned value (so using it waits for all of them).
__device__ __forceinline__ unsigned long long put_low(const TableArgs &t, uint64_t s, u128 k) {
    return xchg(&t.keys[s], (uint64_t)k);
}
__device__ __forceinline__ unsigned long long put_low(const TableArgs &t, uint64_t s,
                                                      const u256 &k) {
    const unsigned long long a = xchg(&t.keys[s], k.w0);
    const unsigned long long b = xchg(&t.keys_mid[2 * s], k.w1);
    const unsigned long long c = xchg(&t.keys_mid[2 * s + 1], k.w2);
    return a ^ b ^ c;
}

// Lower words of slot s equal those of key: device-coherent loads (record)
// or plain loads of a finished table (decision), all issued before any
// comparison so they are in flight together.
__device__ __forceinline__ bool low_equal(const TableArgs &t, uint64_t s, u128 k) {
    return ld(&t.keys[s]) == (uint64_t)k;
}
__device__ __forceinline__ bool low_equal(const TableArgs &t, uint64_t s, const u256 &k) {
    const unsigned long long a = ld(&t.keys[s]), b = ld(&t.keys_mid[2 * s]),
                             c = ld(&t.keys_mid[2 * s + 1]);
    return ((a ^ k.w0) | (b ^ k.w1) | (c ^ k.w2)) == 0;
}
__device__ __forceinline__ bool low_equal_ro(const TableArgs &t, uint64_t s, u128 k) {
    return t.keys[s] == (uint64_t)k;
}
__device__ __forceinline__ bool low_equal_ro(const TableArgs &t, uint64_t s, const u256 &k) {
    const uint64_t a = t.keys[s], b = t.keys_mid[2 * s], c = t.keys_mid[2 * s + 1];
    return ((a ^ k.w0) | (b ^ k.w1) | (c ^ k.w2)) == 0;
}

template <bool P2, class T>
__device__ __forceinline__ int insert_wide(const TableArgs &t, const T &key, uint32_t m,
                                           uint64_t s, unsigned long long cur, uint32_t &visits) {
    const unsigned long long khi = top_word(key);
    int result = 2;  // 2 = in progress, 1 = claimed, 0 = found, -1 = overflow
    uint32_t probes = 0;
    bool reload = false;
    for (uint32_t trip = 0; trip < 4 * MAX_PROBE; ++trip) {
        if (!__any(result == 2))
            break;
        if (result != 2)
            continue;
        ++visits;
        if (reload)
            cur = ld(&t.keys_hi[s]);
        reload = true;
        const uint32_t mw = t.himask ? 0u : ld_mask(t.masks, s);  // issued with the top word
        bool claimed = false;
        if (cur == EMPTY_KEY) {
            const unsigned long long prev = atomicCAS(&t.keys_hi[s], EMPTY_KEY, khi | PENDING_BIT);
            if (prev == EMPTY_KEY)
                claimed = true;
            else
                cur = prev;
        }
        bool advance = false;
        if (claimed) {
            const unsigned long long was = put_low(t, s, key);
            // use the exchanges' results, so they have completed before the publish
            __asm__ volatile("" : : "v"(was));
            if (t.himask) {
                (void)xchg(&t.keys_hi[s], khi | (unsigned long long)m << HIMASK_SHIFT);
            } else {
                (void)xchg(&t.keys_hi[s], khi);
                or_mask(t.masks, s, m, mw);
            }
            result = 1;
        } else if ((cur & (t.himask ? HIKEY_BITS : ~PENDING_BIT)) == khi) {
            // pending: the lower words are not published yet, look again next trip
            if (!(cur & PENDING_BIT)) {
                if (low_equal(t, s, key)) {
                    if (t.himask) {
                        const unsigned long long mm = (unsigned long long)m << HIMASK_SHIFT;
                        if ((cur & mm) != mm)
                            __hip_atomic_fetch_or(&t.keys_hi[s], mm, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        or_mask(t.masks, s, m, mw);
                    }
                    result = 0;
                } else {
                    advance = true;
                }
            }
        } else {
            advance = true;
        }
        if (advance) {
            if (++probes >= MAX_PROBE)
                result = -1;
            else
                s = next_slot<P2>(t, s);
        }
    }
    return result == 2 ? -1 : result;
}

template <bool P2>
__device__ __forceinline__ int insert_from(const TableArgs &t, u128 key, uint32_t m, uint64_t s,
                                           unsigned long long cur, uint32_t &visits) {
    return insert_wide<P2>(t, key, m, s, cur, visits);
}
template <bool P2>
__device__ __forceinline__ int insert_from(const TableArgs &t, const u256 &key, uint32_t m,
                                           uint64_t s, unsigned long long cur,
                                           uint32_t &visits) {
    return insert_wide<P2>(t, key, m, s, cur, visits);
}

// Edge bits of the slot holding key, starting at slot s with word cur, or -1
// when absent.
template <bool P2>
__device__ __forceinline__ int find_from(const TableArgs &t, uint64_t key, uint64_t s,
                                         unsigned long long cur, uint32_t &probes) {
    for (uint32_t i = 0; i < MAX_PROBE; ++i) {
        ++probes;
        if (i)
            cur = t.keys[s];
        if (t.packed) {
            if ((cur >> 8) == key)
                return (int)(cur & 0xFFu);
        } else {
            if (cur == key)
                return mask_byte(t.masks[s >> 2], s);
        }
        if (cur == EMPTY_KEY)
            return -1;
        s = next_slot<P2>(t, s);
    }
    return -1;
}

template <bool P2, class T>
__device__ __forceinline__ int find_wide(const TableArgs &t, const T &key, uint64_t s,
                                         unsigned long long cur, uint32_t &probes) {
    const unsigned long long khi = top_word(key);
    for (uint32_t i = 0; i < MAX_PROBE; ++i) {
        ++probes;
        if (i)
            cur = t.keys_hi[s];
        if (t.himask) {
            if (cur != EMPTY_KEY && (cur & HIKEY_BITS) == khi && low_equal_ro(t, s, key))
                return (int)((cur >> HIMASK_SHIFT) & 0xFFu);
        } else if (cur == khi && low_equal_ro(t, s, key)) {
            return mask_byte(t.masks[s >> 2], s);
        }
        if (cur == EMPTY_KEY)
            return -1;
        s = next_slot<P2>(t, s);
    }
    return -1;
}

template <bool P2>
__device__ __forceinline__ int find_from(const TableArgs &t, u128 key, uint64_t s,
                                         unsigned long long cur, uint32_t &probes) {
    return find_wide<P2>(t, key, s, cur, probes);
}
template <bool P2>
__device__ __forceinline__ int find_from(const TableArgs &t, const u256 &key, uint64_t s,
                                         unsigned long long cur, uint32_t &probes) {
    return find_wide<P2>(t, key, s, cur, probes);
}

// Whether a set's table overflowed in this attempt (thread 0 only): the
// device-coherent flag is read again when the set changes and every 8th
// tile, so the workgroups do not all read one counter line per tile.  A late
// reading only delays the skip; the attempt is redone either way.
__device__ __forceinline__ uint32_t overflow_seen(const SeqArgs &a, uint32_t set,
                                                  uint32_t &flag_set, uint32_t &flag_age,
                                                  uint32_t &flag) {
    if (set != flag_set || (++flag_age & 7) == 0) {
        flag = (uint32_t)__hip_atomic_load(&a.set_cnt[set].overflow, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
        flag_set = set;
        flag_age = 0;
    }
    return flag;
}

// ------------------------------------------------------------- record (a3)

// The normalised k-mer of position p (at offset r of the staged words w) in
// the string [gs, ge), and in m its edge bits: the predecessor's base as an
// in-bit and the successor's as an out-bit, for the orientation in which the
// k-mer is normalised (both orientations for a palindrome).
template <class T>
__device__ __forceinline__ T record_key(const uint64_t *w, uint32_t r, uint32_t k, uint64_t p,
                                        uint64_t gs, uint64_t ge, bool single, uint32_t &m) {
    const Strands<T> st = strands(KT<T>::window(w, r, k), k);
    const bool has_pred = p > gs, has_succ = p + k < ge;
    const uint32_t pa = has_pred ? base_at(w, r - 1) : 0;
    const uint32_t sb = has_succ ? base_at(w, r + k) : 0;
    m = 0;
    T canon = st.fwd;
    if (single || st.fwd <= st.rc) {
        // the k-mer as read is normalised: pred.v enters, v.succ leaves
        if (has_pred)
            m |= 1u << pa;
        if (has_succ)
            m |= 16u << sb;
    }
    if (!single && st.rc <= st.fwd) {
        // its reverse complement is normalised: comp(succ) enters, comp(pred)
        // leaves
        if (has_succ)
            m |= 1u << (3 - sb);
        if (has_pred)
            m |= 16u << (3 - pa);
        canon = st.rc;
    }
    return canon;
}

template <class T, bool P2>
__global__ __launch_bounds__(BLOCK) void k_record(SeqArgs a, const uint64_t *c1, TableArgs pool,
                                                  Counters *cnt) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint64_t cw[TILE / 64];
    __shared__ unsigned long long block_probes, keys_lds;
    __shared__ uint32_t skip_lds;
    uint32_t flag_set = ~0u, flag_age = 0, flag_val = 0;  // thread 0: last flag reading
    SetSum keys = setsum_begin();
    const uint32_t k = a.k;
    const bool single = a.single != 0;
    const bool wide = KT<T>::W >= 2;
    const uint32_t lane = threadIdx.x & 63;
    if (threadIdx.x == 0)
        block_probes = 0;
    uint32_t my_probes = 0;
    // memory order spreads homologous tiles' claims out in time; runs of them
    // on one workgroup keep their slots hot without the concurrent claims of
    // the plain first-pass order
    const uint32_t order = a.pass2_slabs;
    RunCursor rc = (order & 4) ? run_cursor(a, a.chunk > RECORD_RUN ? a.chunk : RECORD_RUN)
                   : (order & 1) ? run_cursor(a, a.chunk) : linear_run(a);
    for (uint64_t tile; run_next(a, rc, &tile);) {
        const uint64_t t0 = tile * TILE;
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        if (lo == hi)
            continue;
        const uint32_t set = ti.set;
        __syncthreads();
        stage_tile2(a, tile, w, c1, cw);
        // a set whose table overflowed in this attempt is redone with a
        // larger table: skip the rest of its work now.  Other workgroups may
        // set the flag at any time, so one thread reads it and the whole
        // workgroup takes that one reading (the skip stays uniform).
        if (threadIdx.x == 0)
            skip_lds = overflow_seen(a, set, flag_set, flag_age, flag_val);
        __syncthreads();
        if (skip_lds)
            continue;
        const TableArgs t = table_of(a, pool, set);
        setsum_switch(keys, set, &keys_lds, &a.set_cnt[0].table_keys, SETCNT_STRIDE);
        bool overflow = false;
        uint64_t gs = ~0ull, ge = 0;  // this lane's last string (positions only grow)
        for (uint32_t it = 0; it < TILE / BLOCK; ++it) {
            const uint64_t p = t0 + it * BLOCK + threadIdx.x;
            if (!((cw[(it * BLOCK + threadIdx.x) >> 6] >> lane) & 1ull))
                continue;
            if (p < gs || p >= ge) {
                const uint32_t si = find_string(a.strings, lo, hi, p);
                if (si == hi)
                    continue;  // not a k-mer start: never marked by the first pass
                gs = a.strings[si].gstart;
                ge = a.strings[si].gend;
            }
            uint32_t m;
            const T canon = record_key<T>(w, (uint32_t)(p - t0) + 32, k, p, gs, ge, single, m);
            const uint64_t slot = first_slot<P2>(t, canon);
            int rc;
            if constexpr (KT<T>::W == 1)
                rc = insert_pair<P2>(t, (uint64_t)canon, m, slot, load_pair(t, slot), my_probes);
            else
                rc = insert_from<P2>(t, canon, m, slot, first_word(t, slot, wide), my_probes);
            if (rc > 0)
                ++keys.v;
            else if (rc < 0)
                overflow = true;
        }
        if (overflow)
            atomicExch(&a.set_cnt[set].overflow, 1ull);
    }
    setsum_flush(keys, &keys_lds, &a.set_cnt[0].table_keys, SETCNT_STRIDE);
    if (my_probes)
        atomicAdd(&block_probes, (unsigned long long)my_probes);
    __syncthreads();
    if (threadIdx.x == 0 && block_probes)
        atomicAdd(&cnt->table_probes, block_probes);
}

hipError_t launch_record(int W, const SeqArgs &a, const uint64_t *c1, const TableArgs &pool,
                         Counters *cnt, uint32_t grid, hipStream_t s) {
    if (a.n_tiles == 0)
        return hipSuccess;
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        if (pool.pow2)
            hipLaunchKernelGGL((k_record<T, true>), dim3(grid), dim3(BLOCK), 0, s, a, c1, pool, cnt);
        else
            hipLaunchKernelGGL((k_record<T, false>), dim3(grid), dim3(BLOCK), 0, s, a, c1, pool,
                               cnt);
        return hipGetLastError();
    });
}

// ------------------------------------------------------ binned record (a3)
//
// The table k_record builds, built block by block instead of by random
// atomics.  A lookup never leaves the block of its home slot (2^e slots,
// e <= TABLE_BLOCK_LOG2), so blocks are independent: a pass takes the blocks
// [r_lo, r_hi); every candidate whose home block is among them becomes an
// item, the slot word it contributes (key << 8 | edge bits, packed slots);
// the items are partitioned by block in two streaming steps (bucket of
// BIN_SUB blocks, then block; each batch sorted in LDS so that a
// destination's items leave as one run); and each block is built in LDS from
// empty and written out whole.  Same keys and edge bits as k_record (slots
// within a block may differ: they follow the order of insertion), no table
// clear and no random access.  Every pass walks the candidates again; the
// passes are as many as the scratch needs.
//
//   k_rbin_count    candidates walked, a static share of the tiles per
//                   workgroup; the pass's items appended to the staging in
//                   segments of RBIN_SEG items that a workgroup claims with
//                   one atomic add (a segment's unused tail holds BIN_NONE)
//   k_rbin_hist     per workgroup (an even share of the staging): items per
//                   bucket
//   k_rbin_scan     offsets per (bucket, workgroup), bucket-major
//   k_rbin_scatter  the same shares, each item to its (bucket, workgroup)
//                   range
//   k_rbin_split    per bucket: its items by block
//   k_rbin_apply    per block: built in LDS, written out; new keys counted

// Home block of a packed slot word (its key is word >> 8).
template <bool P2>
__device__ __forceinline__ uint64_t rbin_block(const TableArgs &t, uint64_t item) {
    return first_slot<P2>(t, item >> 8) >> t.cap_e;
}

template <bool P2>
__global__ __launch_bounds__(BLOCK) void k_rbin_count(SeqArgs a, const uint64_t *c1, TableArgs t,
                                                      RecBinArgs rb) {
    constexpr uint32_t PER = TILE / BLOCK;
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint64_t cw[TILE / 64];
    __shared__ uint32_t wtot[BLOCK / 64];
    __shared__ uint64_t seg_base, seg_new;
    __shared__ uint32_t seg_used;
    const uint32_t k = a.k;
    const bool single = a.single != 0;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        seg_base = 0;
        seg_new = 0;
        seg_used = RBIN_SEG;  // no segment yet
    }
    const uint64_t n = a.n_tiles;
    const uint64_t per = (n + rb.grid - 1) / rb.grid;
    const uint64_t t_lo = min(n, (uint64_t)blockIdx.x * per);
    const uint64_t t_hi = min(n, (uint64_t)(blockIdx.x + 1) * per);
    for (uint64_t tile = t_lo; tile < t_hi; ++tile) {
        const TileInfo ti = a.tiles[tile];
        const uint32_t lo = ti.str_lo, hi = ti.str_hi;
        if (lo == hi)
            continue;
        const uint64_t t0 = tile * TILE;
        __syncthreads();  // the last tile's staged words and segment state are read
        stage_tile2(a, tile, w, c1, cw);
        __syncthreads();
        uint64_t v[PER];
        uint32_t nv = 0;
        uint64_t gs = ~0ull, ge = 0;
#pragma unroll
        for (uint32_t it = 0; it < PER; ++it) {
            v[it] = BIN_NONE;
            const uint64_t p = t0 + it * BLOCK + threadIdx.x;
            if (!((cw[(it * BLOCK + threadIdx.x) >> 6] >> lane) & 1ull))
                continue;
            if (p < gs || p >= ge) {
                const uint32_t si = find_string(a.strings, lo, hi, p);
                if (si == hi)
                    continue;  // not a k-mer start: never marked by the first pass
                gs = a.strings[si].gstart;
                ge = a.strings[si].gend;
            }
            uint32_t m;
            const uint64_t key =
                record_key<uint64_t>(w, (uint32_t)(p - t0) + 32, k, p, gs, ge, single, m);
            const uint64_t item = key << 8 | m;
            const uint64_t r = rbin_block<P2>(t, item);
            if (r >= rb.r_lo && r < rb.r_hi) {
                v[it] = item;
                ++nv;
            }
        }
        // the tile's items in thread order: a scan of the per-thread counts
        uint32_t x = nv;
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d)
                x += y;
        }
        if (lane == 63)
            wtot[wave] = x;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (uint32_t q = 0; q < BLOCK / 64; ++q) {
            before += q < wave ? wtot[q] : 0u;
            total += wtot[q];
        }
        const uint32_t room = RBIN_SEG - seg_used;
        if (threadIdx.x == 0 && total > room) {
            const uint64_t base = atomicAdd(&rb.ctl[0], (unsigned long long)RBIN_SEG);
            seg_new = base;
            if (base + RBIN_SEG > rb.cap)
                atomicExch(&rb.ctl[1], 1ull);
        }
        __syncthreads();
        const uint64_t cur = seg_base + seg_used, nxt = seg_new;
        uint32_t i = before + x - nv;
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            if (v[q] != BIN_NONE) {
                const uint64_t dst = i < room ? cur + i : nxt + (i - room);
                if (dst < rb.cap)
                    rb.items_b[dst] = v[q];
                ++i;
            }
        }
        __syncthreads();  // every thread has read the segment state
        if (threadIdx.x == 0) {
            if (total > room) {
                seg_base = nxt;
                seg_used = total - room;
            } else {
                seg_used += total;
            }
        }
    }
    __syncthreads();
    // the unused tail of the last segment
    for (uint32_t i = seg_used + threadIdx.x; i < RBIN_SEG; i += BLOCK) {
        const uint64_t dst = seg_base + i;
        if (dst < rb.cap)
            rb.items_b[dst] = BIN_NONE;
    }
}

// This workgroup's share of the staging (an even split of what was claimed).
__device__ __forceinline__ void rbin_share(const RecBinArgs &rb, uint64_t *lo, uint64_t *hi) {
    const uint64_t total = min((uint64_t)rb.ctl[0], rb.cap);
    const uint64_t per = (total + rb.grid - 1) / rb.grid;
    *lo = min(total, (uint64_t)blockIdx.x * per);
    *hi = min(total, (uint64_t)(blockIdx.x + 1) * per);
}

template <bool P2>
__global__ __launch_bounds__(BLOCK) void k_rbin_hist(TableArgs t, RecBinArgs rb) {
    __shared__ uint32_t hist[BIN_MAX_BUCKETS];
    for (uint32_t i = threadIdx.x; i < BIN_MAX_BUCKETS; i += BLOCK)
        hist[i] = 0;
    __syncthreads();
    uint64_t lo, hi;
    rbin_share(rb, &lo, &hi);
    if (!rb.ctl[1]) {
        for (uint64_t i = lo + threadIdx.x; i < hi; i += BLOCK) {
            const uint64_t x = rb.items_b[i];
            if (x != BIN_NONE)
                atomicAdd(&hist[(uint32_t)((rbin_block<P2>(t, x) - rb.r_lo) >> BIN_SUB_LOG2)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < rb.n_buckets; i += BLOCK)
        rb.counts[(uint64_t)i * rb.grid + blockIdx.x] = hist[i];
}

__global__ __launch_bounds__(BIN_SCAN_BLOCK) void k_rbin_scan(const uint32_t *counts, uint64_t n,
                                                             uint64_t *offsets) {
    bin_offsets_scan(counts, n, offsets);
}

template <bool P2>
__global__ __launch_bounds__(BIN_SCATTER_BLOCK) void k_rbin_scatter(TableArgs t, RecBinArgs rb) {
    constexpr uint32_t NT = BIN_SCATTER_BLOCK, PER = BIN_SCATTER_PER;
    __shared__ uint64_t cursor[BIN_MAX_BUCKETS];
    __shared__ uint32_t cnt[BIN_MAX_BUCKETS];
    __shared__ uint32_t start[BIN_MAX_BUCKETS];
    __shared__ uint64_t srt[NT * PER];
    __shared__ uint32_t wtot[NT / 64];
    __shared__ uint32_t total;
    for (uint32_t i = threadIdx.x; i < BIN_MAX_BUCKETS; i += NT) {
        cursor[i] = i < rb.n_buckets ? rb.offsets[(uint64_t)i * rb.grid + blockIdx.x] : 0;
        cnt[i] = 0;
    }
    __syncthreads();
    if (rb.ctl[1])
        return;
    uint64_t lo, hi;
    rbin_share(rb, &lo, &hi);
    const auto bucket_of = [&](uint64_t x) {
        return (uint32_t)((rbin_block<P2>(t, x) - rb.r_lo) >> BIN_SUB_LOG2);
    };
    // every thread runs the same number of batches (the workgroup syncs in each)
    for (uint64_t i0 = lo; i0 < hi; i0 += PER * NT) {
        uint64_t v[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint64_t j = i0 + (uint64_t)q * NT + threadIdx.x;
            v[q] = j < hi ? rb.items_b[j] : BIN_NONE;
        }
        sorted_write_by<BIN_MAX_BUCKETS, NT, PER>(v, bucket_of, cnt, start, wtot, &total, srt,
                                                  cursor, rb.items_a);
    }
}

// One workgroup per bucket: its items (the ranges of all its pairs, back to
// back) counted by block, then written block by block into the same range of
// items_b; region_off gets each block's first item.
template <bool P2>
__global__ __launch_bounds__(BIN_SPLIT_BLOCK) void k_rbin_split(TableArgs t, RecBinArgs rb) {
    constexpr uint32_t NT = BIN_SPLIT_BLOCK, PER = BIN_SPLIT_PER;
    __shared__ uint32_t cnt[BIN_SUB];
    __shared__ uint32_t start[BIN_SUB];
    __shared__ uint64_t cursor[BIN_SUB];
    __shared__ uint64_t srt[NT * PER];
    __shared__ uint32_t wtot[NT / 64];
    __shared__ uint32_t total;
    const uint32_t bk = blockIdx.x;
    const uint64_t lo = rb.offsets[(uint64_t)bk * rb.grid];
    const uint64_t hi = rb.offsets[(uint64_t)(bk + 1) * rb.grid];
    const auto sub_of = [&](uint64_t x) {
        return (uint32_t)(rbin_block<P2>(t, x) - rb.r_lo) & (BIN_SUB - 1);
    };
    for (uint32_t i = threadIdx.x; i < BIN_SUB; i += NT)
        cnt[i] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += NT)
        atomicAdd(&cnt[sub_of(rb.items_a[i])], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t c = lo;
        for (uint32_t q = 0; q < BIN_SUB; ++q) {
            cursor[q] = c;
            rb.region_off[(uint64_t)bk * BIN_SUB + q] = c;
            c += cnt[q];
            cnt[q] = 0;
        }
        if (bk + 1 == rb.n_buckets)
            rb.region_off[(uint64_t)rb.n_buckets * BIN_SUB] = c;
    }
    __syncthreads();
    for (uint64_t i0 = lo; i0 < hi; i0 += PER * NT) {
        uint64_t v[PER];
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint64_t j = i0 + (uint64_t)q * NT + threadIdx.x;
            v[q] = j < hi ? rb.items_a[j] : BIN_NONE;
        }
        sorted_write_by<BIN_SUB, NT, PER>(v, sub_of, cnt, start, wtot, &total, srt, cursor,
                                          rb.items_b);
    }
}

// One workgroup per block of the pass: the block built in LDS from empty (an
// item claims an empty slot by compare-and-swap, or ORs its edge bits into
// its key's slot; probes wrap within the block), then written out whole.
template <bool P2>
__global__ __launch_bounds__(BIN_APPLY_BLOCK) void k_rbin_apply(TableArgs t, RecBinArgs rb,
                                                                SetCounters *sc, Counters *cnt) {
    constexpr uint32_t NT = BIN_APPLY_BLOCK;
    __shared__ __align__(16) unsigned long long reg[1u << TABLE_BLOCK_LOG2];
    __shared__ unsigned long long fresh_wg, probes_wg;
    __shared__ uint32_t over_wg;
    const uint32_t nb = 1u << t.cap_e;  // slots per block
    const uint64_t r = blockIdx.x;
    ulonglong2 *reg2 = (ulonglong2 *)reg;
    for (uint32_t i = threadIdx.x; i < nb / 2; i += NT)
        reg2[i] = make_ulonglong2(EMPTY_KEY, EMPTY_KEY);
    if (threadIdx.x == 0) {
        fresh_wg = probes_wg = 0;
        over_wg = 0;
    }
    __syncthreads();
    if (rb.ctl[1])
        return;  // the scratch was too small: the host redoes the record
    const uint64_t lo = rb.region_off[r], hi = rb.region_off[r + 1];
    uint32_t fresh = 0, probes = 0;
    bool over = false;
    constexpr uint32_t U = 4;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += U * NT) {
        uint64_t v[U];
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            const uint64_t j = i + (uint64_t)q * NT;
            v[q] = j < hi ? rb.items_b[j] : BIN_NONE;
        }
#pragma unroll
        for (uint32_t q = 0; q < U; ++q) {
            if (v[q] == BIN_NONE)
                continue;
            const uint64_t key = v[q] >> 8;
            const unsigned long long m = v[q] & 0xFFu;
            uint32_t s = (uint32_t)first_slot<P2>(t, key) & (nb - 1);
            ++probes;
            uint32_t j = 0;
            for (; j < MAX_PROBE; ++j) {
                const unsigned long long cur =
                    atomicCAS(&reg[s], EMPTY_KEY, (unsigned long long)v[q]);
                if (cur == EMPTY_KEY) {
                    ++fresh;
                    break;
                }
                if ((cur >> 8) == key) {
                    if ((cur & m) != m)
                        atomicOr(&reg[s], m);
                    break;
                }
                s = (s + 1) & (nb - 1);
                probes += (s & 1) == 0;  // a new pair of slots
            }
            over |= j == MAX_PROBE;
        }
    }
    if (fresh)
        atomicAdd(&fresh_wg, (unsigned long long)fresh);
    if (probes)
        atomicAdd(&probes_wg, (unsigned long long)probes);
    if (over)
        over_wg = 1;
    __syncthreads();
    ulonglong2 *dst = (ulonglong2 *)(t.keys + ((rb.r_lo + r) << t.cap_e));
    for (uint32_t i = threadIdx.x; i < nb / 2; i += NT)
        dst[i] = reg2[i];
    if (threadIdx.x == 0) {
        if (fresh_wg)
            atomicAdd(&sc->table_keys, fresh_wg);
        if (probes_wg)
            atomicAdd(&cnt->table_probes, probes_wg);
        if (over_wg)
            atomicExch(&sc->overflow, 1ull);
    }
}

hipError_t launch_record_binned(const SeqArgs &a, const uint64_t *c1, const TableArgs &t,
                                RecBinArgs rb, uint32_t passes, uint64_t n_blocks,
                                SetCounters *set_cnt, Counters *cnt, hipStream_t s) {
    if (n_blocks == 0 || passes == 0)
        return hipSuccess;
    hipError_t e = launch_zero(rb.ctl, 2 * sizeof(unsigned long long), s);
    if (e != hipSuccess)
        return e;
    const uint64_t per_pass = (n_blocks + passes - 1) / passes;
    auto run = [&](auto p2) -> hipError_t {
        constexpr bool P2 = decltype(p2)::value;
        for (uint64_t r0 = 0; r0 < n_blocks; r0 += per_pass) {
            rb.r_lo = r0;
            rb.r_hi = min(n_blocks, r0 + per_pass);
            rb.n_buckets = (uint32_t)((rb.r_hi - rb.r_lo + BIN_SUB - 1) / BIN_SUB);
            if (r0) {
                e = launch_zero(rb.ctl, sizeof(unsigned long long), s);  // staging cursor
                if (e != hipSuccess)
                    return e;
            }
            hipLaunchKernelGGL(k_rbin_count<P2>, dim3(rb.grid), dim3(BLOCK), 0, s, a, c1, t, rb);
            hipLaunchKernelGGL(k_rbin_hist<P2>, dim3(rb.grid), dim3(BLOCK), 0, s, t, rb);
            hipLaunchKernelGGL(k_rbin_scan, dim3(1), dim3(BIN_SCAN_BLOCK), 0, s, rb.counts,
                               (uint64_t)rb.n_buckets * rb.grid, rb.offsets);
            hipLaunchKernelGGL(k_rbin_scatter<P2>, dim3(rb.grid), dim3(BIN_SCATTER_BLOCK), 0, s, t,
                               rb);
            hipLaunchKernelGGL(k_rbin_split<P2>, dim3(rb.n_buckets), dim3(BIN_SPLIT_BLOCK), 0, s,
                               t, rb);
            hipLaunchKernelGGL(k_rbin_apply<P2>, dim3((uint32_t)(rb.r_hi - rb.r_lo)),
                               dim3(BIN_APPLY_BLOCK), 0, s, t, rb, set_cnt, cnt);
            e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    return t.pow2 ? run(std::true_type{}) : run(std::false_type{});
}

// ------------------------------------------------------------- decide (a4)

// Lookups a decision thread keeps in flight at once: two one-word keys (a
// pair of slots each), one wide key (whose compare needs its lower words
// after the top word).
template <class T> struct DecideGroup {
    static constexpr uint32_t N = KT<T>::W == 1 ? 2 : 1;
};

// One-word lookup by slot pairs: pr holds the words of slots s and s + 1 (s
// even); the next pair is loaded with one 16-byte read when the key lies
// further on.  Edge bits of the key's slot, or -1 when absent.
template <bool P2>
__device__ __forceinline__ int find_pair(const TableArgs &t, uint64_t key, uint64_t s, u64x2 pr,
                                         uint32_t &probes) {
    for (uint32_t i = 0; i < MAX_PROBE / 2; ++i) {
        if (i)
            pr = load_pair(t, s);
        ++probes;
#pragma unroll
        for (uint32_t half = 0; half < 2; ++half) {
            const unsigned long long w = half ? pr.y : pr.x;
            if (t.packed) {
                if ((w >> 8) == key)
                    return (int)(w & 0xFFu);
            } else if (w == key) {
                return mask_byte(t.masks[(s + half) >> 2], s + half);
            }
            if (w == EMPTY_KEY)
                return -1;
        }
        s = next_pair<P2>(t, s);
    }
    return -1;
}

template <class T, bool P2>
__global__ __launch_bounds__(BLOCK) void k_decide(SeqArgs a, SentArgs sa, const uint64_t *c1,
                                                  TableArgs pool, uint64_t *jbits,
                                                  bool accumulate, Counters *cnt) {
    __shared__ uint64_t w[STAGE_WORDS];
    __shared__ uint64_t cw[TILE / 64];
    __shared__ uint32_t pf[(1u << PF_MAX_LOG2) / 32];
    __shared__ unsigned long long block_probes, junc_lds;
    __shared__ uint32_t skip_lds;
    uint32_t flag_set = ~0u, flag_age = 0, flag_val = 0;  // thread 0: last flag reading
    SetSum junc = setsum_begin();
    const uint32_t k = a.k;
    const bool single = a.single != 0;
    const bool wide = KT<T>::W >= 2;
    const T *sent = (const T *)sa.table;
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t i = threadIdx.x; i < (1u << sa.pf_log2) / 32; i += BLOCK)
        pf[i] = sa.prefilter[i];
    if (threadIdx.x == 0)
        block_probes = 0;
    unsigned long long my_missing = 0;
    uint32_t my_probes = 0;
    // homologous tiles at once (slab order) share table lines in L2; lookups
    // do not contend, unlike the record's atomics
    RunCursor rc = (a.pass2_slabs & 2) ? run_cursor(a, a.chunk) : linear_run(a);
    for (uint64_t tile; run_next(a, rc, &tile);) {
        const uint64_t t0 = tile * TILE;
        const uint32_t set = a.tiles[tile].set;
        __syncthreads();
        stage_tile2(a, tile, w, c1, cw);
        if (threadIdx.x == 0)
            skip_lds = overflow_seen(a, set, flag_set, flag_age, flag_val);
        __syncthreads();
        if (skip_lds) {
            // this attempt's table overflowed: its results are discarded (the
            // run is redone, or reports the overflow); the tile's junction
            // words are still defined
            if (!accumulate && threadIdx.x < TILE / 64)
                jbits[tile * (TILE / 64) + threadIdx.x] = 0;
            continue;
        }
        const TableArgs t = table_of(a, pool, set);
        const SetDesc &sd = a.sets[set];
        const T *stab = sent + sd.sent_tab_off;
        const uint32_t slog2 = sd.sent_tab_log2;
        setsum_switch(junc, set, &junc_lds, &a.set_cnt[0].junctions, SETCNT_STRIDE);
        // A thread's positions of the tile in groups: the group's candidate
        // k-mers and home slots are computed from LDS alone, then every table
        // word (and, on a sentinel-prefilter hit, the sentinel-table word) is
        // loaded at once, so that many random reads are in flight per lane
        // before any is needed; then each lookup is resolved.
        for (uint32_t g0 = 0; g0 < TILE / BLOCK; g0 += DecideGroup<T>::N) {
            constexpr uint32_t G = DecideGroup<T>::N;
            constexpr bool ONE = KT<T>::W == 1;
            T canon[G];
            uint64_t slot[G];
            u64x2 cur[G];
            uint32_t ss[G];
            T sx[G];
            uint32_t look = 0, maybe_sent = 0, junction = 0;
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                const uint32_t q = (g0 + j) * BLOCK + threadIdx.x;  // position in the tile
                canon[j] = 0;
                slot[j] = 0;
                ss[j] = 0;
                if ((cw[q >> 6] >> lane) & 1ull) {
                    canon[j] = norm(strands(KT<T>::window(w, q + 32, k), k), single);
                    look |= 1u << j;
                    slot[j] = first_slot<P2>(t, canon[j]);
                    if (slog2 && prefilter_hit(canon[j], pf, sa.pf_log2)) {
                        maybe_sent |= 1u << j;
                        ss[j] = sent_home(canon[j], slog2);
                    }
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                cur[j].x = cur[j].y = 0;
                if ((look >> j) & 1u) {
                    if (ONE)
                        cur[j] = load_pair(t, slot[j]);
                    else
                        cur[j].x = first_word_ro(t, slot[j], wide);
                }
                sx[j] = ((maybe_sent >> j) & 1u) ? stab[ss[j]] : T(0);
            }
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                if (!((look >> j) & 1u))
                    continue;
                if (((maybe_sent >> j) & 1u) &&
                    sent_probe_from(stab, slog2, canon[j], ss[j], sx[j])) {
                    junction |= 1u << j;  // a sentinel k-mer
                    continue;
                }
                int m;
                if constexpr (ONE)
                    m = find_pair<P2>(t, (uint64_t)canon[j], slot[j], cur[j], my_probes);
                else
                    m = find_from<P2>(t, canon[j], slot[j], cur[j].x, my_probes);
                if (m < 0)
                    ++my_missing;
                else if (__popc((uint32_t)m & 15u) > 1 || __popc((uint32_t)m >> 4) > 1)
                    junction |= 1u << j;
            }
#pragma unroll
            for (uint32_t j = 0; j < G; ++j) {
                const uint64_t p = t0 + (g0 + j) * BLOCK + threadIdx.x;
                const uint64_t jw = ballot64((junction >> j) & 1u);
                if (lane == 0) {
                    jbits[p >> 6] = accumulate ? jbits[p >> 6] | jw : jw;
                    junc.v += (unsigned long long)__popcll(jw);
                }
            }
        }
    }
    setsum_flush(junc, &junc_lds, &a.set_cnt[0].junctions, SETCNT_STRIDE);
    if (my_probes)
        atomicAdd(&block_probes, (unsigned long long)my_probes);
    if (my_missing)
        atomicAdd(&cnt->missing, my_missing);
    __syncthreads();
    if (threadIdx.x == 0 && block_probes)
        atomicAdd(&cnt->table_probes, block_probes);
}

// Resident workgroups per CU of both table modes' instantiations (the fewer).
hipError_t pass2_occupancy(KernelId which, int W, int *blocks) {
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        const void *fn[2] = {
            which == K_RECORD ? (const void *)k_record<T, true> : (const void *)k_decide<T, true>,
            which == K_RECORD ? (const void *)k_record<T, false> : (const void *)k_decide<T, false>};
        int n[2] = {0, 0};
        for (int i = 0; i < 2; ++i) {
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n[i], fn[i], BLOCK, 0);
            if (e != hipSuccess)
                return e;
        }
        *blocks = std::min(n[0], n[1]);
        return hipSuccess;
    });
}

hipError_t launch_decide(int W, const SeqArgs &a, const SentArgs &sa, const uint64_t *c1,
                         const TableArgs &pool, uint64_t *jbits, bool accumulate, Counters *cnt,
                         uint32_t grid, hipStream_t s) {
    if (a.n_tiles == 0)
        return hipSuccess;
    return by_width(W, [&](auto tag) {
        using T = decltype(tag);
        if (pool.pow2)
            hipLaunchKernelGGL((k_decide<T, true>), dim3(grid), dim3(BLOCK), 0, s, a, sa, c1, pool,
                               jbits, accumulate, cnt);
        else
            hipLaunchKernelGGL((k_decide<T, false>), dim3(grid), dim3(BLOCK), 0, s, a, sa, c1,
                               pool, jbits, accumulate, cnt);
        return hipGetLastError();
    });
}

}  // namespace tp
