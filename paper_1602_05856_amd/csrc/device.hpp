// Device helpers of the gfx950 junction-finding kernels: k-mer windows read
// from 2-bit packed sequence staged in LDS, normalised (canonical) k-mers,
// the Bloom/table hash specification, string (contig) lookup and the
// sentinel filter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"

namespace tp {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- hash spec
// mix64 is the SplitMix64 output function (Steele, Lea & Flood 2014).
// Bloom bit t of a normalised (k+1)-mer e: (H1 + t*H2) mod 2^64 mod b with
// H1 = mix64(fold(e) ^ S1), H2 = mix64(fold(e) ^ S2) | 1 (double hashing,
// Kirsch & Mitzenmacher 2006).  fold(e) = e for one-word values, else
// mix64(hi ^ S0) ^ lo.  Table slot of a normalised k-mer v:
// mix64(fold(v) ^ S3) mod capacity.  S0..S3 are hexadecimal digits of pi.
constexpr uint64_t kS0 = 0x243F6A8885A308D3ull;
constexpr uint64_t kS1 = 0x13198A2E03707344ull;
constexpr uint64_t kS2 = 0xA4093822299F31D0ull;
constexpr uint64_t kS3 = 0x082EFA98EC4E6C89ull;
constexpr uint64_t kS4 = 0x452821E638D01377ull;  // k-mer classes (multiple rounds)

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Reverse the order of the 2-bit groups of a 64-bit word.
__device__ __forceinline__ uint64_t rev2(uint64_t x) {
    uint64_t y = __builtin_bitreverse64(x);
    return ((y >> 1) & 0x5555555555555555ull) | ((y & 0x5555555555555555ull) << 1);
}

// (lo >> sh) | (hi << (64 - sh)) for 0 <= sh < 64, without a branch.
__device__ __forceinline__ uint64_t funnel(uint64_t lo, uint64_t hi, uint32_t sh) {
    return (lo >> sh) | ((hi << 1) << (63 - sh));
}

// Four-word unsigned value (k <= 127: up to 128 bases), w0 least
// significant, with the operators the k-mer code uses.  Shifts by a variable
// count select words with conditional moves (no indexed register arrays).
struct u256 {
    uint64_t w0, w1, w2, w3;
    u256() = default;
    __host__ __device__ constexpr u256(uint64_t x) : w0(x), w1(0), w2(0), w3(0) {}
    __host__ __device__ constexpr u256(uint64_t a, uint64_t b, uint64_t c, uint64_t d)
        : w0(a), w1(b), w2(c), w3(d) {}
    __device__ __forceinline__ explicit operator uint64_t() const { return w0; }
    __device__ __forceinline__ explicit operator uint32_t() const { return (uint32_t)w0; }
};

__device__ __forceinline__ uint64_t u256_word(const u256 &a, uint32_t i) {
    return i == 0 ? a.w0 : i == 1 ? a.w1 : i == 2 ? a.w2 : i == 3 ? a.w3 : 0ull;
}
__device__ __forceinline__ u256 operator>>(const u256 &a, uint32_t n) {
    if (n >= 256)
        return u256(0);
    const uint32_t q = n >> 6, sh = n & 63;
    auto part = [&](uint32_t i) {
        const uint64_t lo = u256_word(a, i + q), hi = u256_word(a, i + q + 1);
        return sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
    };
    return u256(part(0), part(1), part(2), part(3));
}
__device__ __forceinline__ u256 operator<<(const u256 &a, uint32_t n) {
    if (n >= 256)
        return u256(0);
    const uint32_t q = n >> 6, sh = n & 63;
    auto part = [&](uint32_t i) {
        const uint64_t hi = i >= q ? u256_word(a, i - q) : 0ull;
        const uint64_t lo = i >= q + 1 ? u256_word(a, i - q - 1) : 0ull;
        return sh ? (hi << sh) | (lo >> (64 - sh)) : hi;
    };
    return u256(part(0), part(1), part(2), part(3));
}
__device__ __forceinline__ u256 operator&(const u256 &a, const u256 &b) {
    return u256(a.w0 & b.w0, a.w1 & b.w1, a.w2 & b.w2, a.w3 & b.w3);
}
__device__ __forceinline__ u256 operator|(const u256 &a, const u256 &b) {
    return u256(a.w0 | b.w0, a.w1 | b.w1, a.w2 | b.w2, a.w3 | b.w3);
}
__device__ __forceinline__ u256 operator^(const u256 &a, const u256 &b) {
    return u256(a.w0 ^ b.w0, a.w1 ^ b.w1, a.w2 ^ b.w2, a.w3 ^ b.w3);
}
__device__ __forceinline__ u256 operator~(const u256 &a) {
    return u256(~a.w0, ~a.w1, ~a.w2, ~a.w3);
}
__device__ __forceinline__ bool operator==(const u256 &a, const u256 &b) {
    return ((a.w0 ^ b.w0) | (a.w1 ^ b.w1) | (a.w2 ^ b.w2) | (a.w3 ^ b.w3)) == 0;
}
__device__ __forceinline__ bool operator!=(const u256 &a, const u256 &b) { return !(a == b); }
__device__ __forceinline__ bool operator<(const u256 &a, const u256 &b) {
    if (a.w3 != b.w3)
        return a.w3 < b.w3;
    if (a.w2 != b.w2)
        return a.w2 < b.w2;
    if (a.w1 != b.w1)
        return a.w1 < b.w1;
    return a.w0 < b.w0;
}
__device__ __forceinline__ bool operator>(const u256 &a, const u256 &b) { return b < a; }
__device__ __forceinline__ bool operator<=(const u256 &a, const u256 &b) { return !(b < a); }
__device__ __forceinline__ bool operator>=(const u256 &a, const u256 &b) { return !(a < b); }

// Host-side dispatch on the k-mer width: f(tag) with a value of the k-mer
// type of W words (1: uint64_t, 2: u128, 4: u256).
template <class F> hipError_t by_width(int W, F &&f) {
    if (W == 1)
        return f(uint64_t{});
    if (W == 2)
        return f(u128{});
    return f(u256{});
}

// k-mer word traits: W = 1 (uint64_t, k <= 31), W = 2 (u128, k <= 63) or
// W = 4 (u256, k <= 127).  fold(x): the top word, then for each lower word
// f = mix64(f ^ S0) ^ word.
template <class T> struct KT;

template <> struct KT<uint64_t> {
    static constexpr int W = 1;
    __device__ static __forceinline__ uint64_t fold(uint64_t x) { return x; }
    __device__ static __forceinline__ uint64_t ones(uint32_t nbits) {
        return nbits >= 64 ? ~0ull : ((1ull << nbits) - 1);
    }
    // LSB-first window of L <= 32 bases starting at base index r of words w.
    __device__ static __forceinline__ uint64_t window(const uint64_t *w, uint32_t r, uint32_t L) {
        uint32_t q = r >> 5, sh = 2 * (r & 31);
        return funnel(w[q], w[q + 1], sh) & ones(2 * L);
    }
    // val (first base most significant) of an LSB-first window of L bases.
    __device__ static __forceinline__ uint64_t val(uint64_t x, uint32_t L) {
        return rev2(x) >> (64 - 2 * L);
    }
    __device__ static __forceinline__ uint64_t lo(uint64_t x) { return x; }
    __device__ static __forceinline__ uint64_t hi(uint64_t) { return 0; }
    __device__ static __forceinline__ uint64_t word(uint64_t x, uint32_t) { return x; }
};

template <> struct KT<u128> {
    static constexpr int W = 2;
    __device__ static __forceinline__ uint64_t fold(u128 x) {
        return mix64((uint64_t)(x >> 64) ^ kS0) ^ (uint64_t)x;
    }
    __device__ static __forceinline__ u128 ones(uint32_t nbits) {
        return nbits >= 128 ? ~(u128)0 : (((u128)1 << nbits) - 1);
    }
    __device__ static __forceinline__ u128 window(const uint64_t *w, uint32_t r, uint32_t L) {
        uint32_t q = r >> 5, sh = 2 * (r & 31);
        uint64_t a = funnel(w[q], w[q + 1], sh);
        uint64_t b = funnel(w[q + 1], w[q + 2], sh);
        return (((u128)b << 64) | a) & ones(2 * L);
    }
    __device__ static __forceinline__ u128 val(u128 x, uint32_t L) {
        u128 r = ((u128)rev2((uint64_t)x) << 64) | rev2((uint64_t)(x >> 64));
        return r >> (128 - 2 * L);
    }
    __device__ static __forceinline__ uint64_t lo(u128 x) { return (uint64_t)x; }
    __device__ static __forceinline__ uint64_t hi(u128 x) { return (uint64_t)(x >> 64); }
    __device__ static __forceinline__ uint64_t word(u128 x, uint32_t i) {
        return i == 0 ? (uint64_t)x : (uint64_t)(x >> 64);
    }
};

template <> struct KT<u256> {
    static constexpr int W = 4;
    __device__ static __forceinline__ uint64_t fold(const u256 &x) {
        uint64_t f = x.w3;
        f = mix64(f ^ kS0) ^ x.w2;
        f = mix64(f ^ kS0) ^ x.w1;
        return mix64(f ^ kS0) ^ x.w0;
    }
    __device__ static __forceinline__ u256 ones(uint32_t nbits) {
        auto part = [&](uint32_t i) -> uint64_t {
            const uint32_t lo = 64 * i;
            return nbits >= lo + 64 ? ~0ull : nbits <= lo ? 0ull : ((1ull << (nbits - lo)) - 1);
        };
        return u256(part(0), part(1), part(2), part(3));
    }
    // LSB-first window of L <= 128 bases starting at base index r of words w.
    __device__ static __forceinline__ u256 window(const uint64_t *w, uint32_t r, uint32_t L) {
        const uint32_t q = r >> 5, sh = 2 * (r & 31);
        const u256 x(funnel(w[q], w[q + 1], sh), funnel(w[q + 1], w[q + 2], sh),
                     funnel(w[q + 2], w[q + 3], sh), funnel(w[q + 3], w[q + 4], sh));
        return x & ones(2 * L);
    }
    __device__ static __forceinline__ u256 val(const u256 &x, uint32_t L) {
        const u256 r(rev2(x.w3), rev2(x.w2), rev2(x.w1), rev2(x.w0));
        return r >> (256 - 2 * L);
    }
    __device__ static __forceinline__ uint64_t lo(const u256 &x) { return x.w0; }
    __device__ static __forceinline__ uint64_t hi(const u256 &x) { return x.w1; }
    __device__ static __forceinline__ uint64_t word(const u256 &x, uint32_t i) {
        return u256_word(x, i);
    }
};

// The value and reverse-complement value of an L-mer given its LSB-first
// window x: the reverse complement of base string s is sum (3-s[t]) 4^t over
// the LSB-first order, i.e. x with every 2-bit group complemented.
template <class T> struct Strands {
    T fwd, rc;
};

template <class T>
__device__ __forceinline__ Strands<T> strands(T x, uint32_t L) {
    Strands<T> s;
    s.fwd = KT<T>::val(x, L);
    s.rc = x ^ KT<T>::ones(2 * L);
    return s;
}

template <class T>
__device__ __forceinline__ T norm(const Strands<T> &s, bool single) {
    return (single || s.fwd <= s.rc) ? s.fwd : s.rc;
}

// Base code at base index r of words w.
__device__ __forceinline__ uint32_t base_at(const uint64_t *w, uint32_t r) {
    return (uint32_t)(w[r >> 5] >> (2 * (r & 31))) & 3u;
}

// --------------------------------------------------------------- Bloom ops
struct BloomHash {
    uint64_t h1, h2;
};

template <class T>
__device__ __forceinline__ BloomHash bloom_hash(T e) {
    uint64_t f = KT<T>::fold(e);
    BloomHash bh;
    bh.h1 = mix64(f ^ kS1);
    bh.h2 = mix64(f ^ kS2) | 1ull;
    return bh;
}

// Blocked filter: all h bits of an edge x.m.y lie in the 64-bit block of its
// normalised middle (k-1)-mer mu: block = mix64(fold(mu) ^ S1) mod (b/64);
// with G = mix64(fold(mu) ^ S2), a = G & 63, d = ((G >> 6) & 63) | 1, the edge
// written in mu's orientation as (p, q) sets bits (a + (j*h + t)*d) mod 64,
// j = 4p + q, t < h.  orient: 0 middle read forward, 1 middle reversed,
// 2 palindromic middle (orientation of the normalised edge decides).
struct MiddleKey {
    uint64_t block;
    uint64_t g;  // G (also an orientation-free hash of the middle)
    uint32_t a, d, orient;
};

template <class T>
__device__ __forceinline__ MiddleKey middle_key(T mf, T mr, bool single, uint64_t nblock_mask) {
    T mu;
    MiddleKey key;
    if (single || mf < mr) {
        mu = mf;
        key.orient = 0;
    } else if (mf > mr) {
        mu = mr;
        key.orient = 1;
    } else {
        mu = mf;
        key.orient = 2;
    }
    const uint64_t f = KT<T>::fold(mu);
    key.block = mix64(f ^ kS1) & nblock_mask;
    const uint64_t g = mix64(f ^ kS2);
    key.g = g;
    key.a = (uint32_t)(g & 63);
    key.d = (uint32_t)((g >> 6) & 63) | 1u;
    return key;
}

// Bits of edge pair j = 4p + q inside its block.
__device__ __forceinline__ uint64_t pair_mask(uint32_t a, uint32_t d, uint32_t j, uint32_t h) {
    uint64_t m = 0;
    for (uint32_t t = 0; t < h; ++t)
        m |= 1ull << ((a + (j * h + t) * d) & 63u);
    return m;
}

// Pair index of edge x.m.y in its middle's orientation; fwd_le_rc tells
// whether val(edge) <= val(rc(edge)) (used for palindromic middles only).
__device__ __forceinline__ uint32_t pair_index(uint32_t orient, uint32_t x, uint32_t y,
                                               bool fwd_le_rc) {
    const bool flip = orient == 1 || (orient == 2 && !fwd_le_rc);
    return flip ? 4 * (3 - y) + (3 - x) : 4 * x + y;
}

template <class T>
__device__ __forceinline__ uint64_t slot_hash(T v) {
    return mix64(KT<T>::fold(v) ^ kS3);
}

// Class subrange of a normalised k-mer for the multiple-rounds partition
// (Multiple Rounds section): the top CLASS_Q_LOG2 bits of mix64(fold(v) ^ S4).
template <class T>
__device__ __forceinline__ uint32_t class_subrange(T v) {
    return (uint32_t)(mix64(KT<T>::fold(v) ^ kS4) >> (64 - CLASS_Q_LOG2));
}

__device__ __forceinline__ bool in_class(uint32_t sub, uint32_t lo, uint32_t hi) {
    return sub >= lo && sub < hi;
}

// Normalised k-mers at p and p + 1 of the (k+1)-mer e at p: the prefix reads
// fwd >> 2 forward and rc & ones(2k) reversed, the suffix fwd & ones(2k) and
// rc >> 2.
template <class T>
__device__ __forceinline__ void edge_kmers(const Strands<T> &e, uint32_t k, bool single, T *pre,
                                           T *suf) {
    const T ones = KT<T>::ones(2 * k);
    Strands<T> a, b;
    a.fwd = e.fwd >> 2;
    a.rc = e.rc & ones;
    b.fwd = e.fwd & ones;
    b.rc = e.rc >> 2;
    *pre = norm(a, single);
    *suf = norm(b, single);
}

// ---------------------------------------------------------- string lookup
// Strings (contigs) of length >= k, sorted by gstart, disjoint, in global
// base-index coordinates.  find the last string with gstart <= p among
// [lo, hi); returns hi when there is none.
__device__ __forceinline__ uint32_t find_string(const DString *S, uint32_t lo, uint32_t hi,
                                                uint64_t p) {
    uint32_t a = lo, b = hi;  // answer in [a-1, b)
    while (a < b) {
        uint32_t m = (a + b) >> 1;
        if (S[m].gstart <= p)
            a = m + 1;
        else
            b = m;
    }
    return a == lo ? hi : a - 1;
}

// ------------------------------------------------------- sentinel filter
// Sentinel k-mers (normalised first and last k-mer of every string): a bit
// prefilter kept in LDS, then the set's open-addressing sentinel table.
constexpr uint64_t kS6 = 0xC0AC29B7C97C50DDull;  // sentinel-table slots

template <class T>
__device__ __forceinline__ uint32_t prefilter_bit(T v, uint32_t log2bits) {
    return (uint32_t)((KT<T>::fold(v) * 0x9E3779B97F4A7C15ull) >> (64 - log2bits));
}

template <class T>
__device__ __forceinline__ bool prefilter_hit(T v, const uint32_t *lds_pf, uint32_t log2bits) {
    const uint32_t bit = prefilter_bit(v, log2bits);
    return (lds_pf[bit >> 5] >> (bit & 31)) & 1u;
}

// Home slot of v in a sentinel table of 2^log2 slots.
template <class T>
__device__ __forceinline__ uint32_t sent_home(T v, uint32_t log2) {
    return (uint32_t)(mix64(KT<T>::fold(v) ^ kS6) >> (64 - log2));
}

// Whether v is in the sentinel table tab[0 .. 2^log2), probing from slot s
// whose value x has already been read.  The table is at most half full, so
// an empty slot ends every probe sequence.
template <class T>
__device__ __forceinline__ bool sent_probe_from(const T *tab, uint32_t log2, T v, uint32_t s, T x) {
    const uint32_t mask = (1u << log2) - 1;
    for (uint32_t i = 0; i <= mask; ++i) {
        if (i)
            x = tab[s];
        if (x == v)
            return true;
        if (x == ~T(0))
            return false;
        s = (s + 1) & mask;
    }
    return false;
}

// Membership in a set's sentinel table (tab: the set's first slot).
template <class T>
__device__ __forceinline__ bool is_sentinel(T v, const uint32_t *lds_pf, uint32_t pf_log2,
                                            const T *tab, uint32_t log2) {
    if (!log2 || !prefilter_hit(v, lds_pf, pf_log2))
        return false;
    const uint32_t s = sent_home(v, log2);
    return sent_probe_from(tab, log2, v, s, tab[s]);
}

// A tile's set: its index, sentinel slice and filter region.
struct TileSet {
    uint32_t set;
    uint32_t sent_log2;
    uint64_t sent_off;
    uint32_t cls_lo, cls_hi;
    BloomArgs f;
};

__device__ __forceinline__ TileSet tile_set_of(const SeqArgs &a, const BloomArgs &pool,
                                               uint32_t set) {
    TileSet ts;
    ts.set = set;
    const SetDesc &d = a.sets[ts.set];
    ts.sent_log2 = d.sent_tab_log2;
    ts.sent_off = d.sent_tab_off;
    ts.cls_lo = d.cls_lo;
    ts.cls_hi = d.cls_hi;
    ts.f = pool;
    ts.f.words = pool.words + d.bloom_off;
    ts.f.mask = d.bloom_mask;
    return ts;
}

// Persistent-grid walks over a workgroup's tiles, in chunks of G
// consecutive entries (the chunk size, tp_config.chunk_tiles): workgroup i
// runs on XCD i mod NXCD (round-robin dispatch) and walks that XCD's share
// of the first-pass tile order (run_cursor), or the tiles in memory order
// (linear_run).  The grid is a multiple of NXCD.  Static schedule: every
// (grid/NXCD)-th chunk of the share, or every grid-th chunk in memory order.
// With a tile queue (SeqArgs.queue): a workgroup takes the next chunk from
// its share's counter (one per XCD; one in memory order) when it finishes
// one, and once that share is exhausted from the other XCDs' shares in
// turn, so the last chunks go to whichever workgroups are free.  The walk is
// the same for every thread of a workgroup; with a queue, every thread must
// call run_next (it synchronises the workgroup to share each claim).
struct RunCursor {
    uint64_t c, end;
    uint32_t gi, G, step, ordered;
    uint32_t qx, qleft;  // queue: the share being walked, shares not yet exhausted
};

__device__ __forceinline__ RunCursor run_cursor(const SeqArgs &a, uint32_t G) {
    const uint32_t x = blockIdx.x % NXCD;
    if (a.queue)  // nothing claimed yet: the first run_next claims
        return RunCursor{0, 0, G, G, 0, 1, x, NXCD};
    return RunCursor{a.xcd_start[x] + (uint64_t)(blockIdx.x / NXCD) * G, a.xcd_start[x + 1], 0,
                     G, gridDim.x / NXCD, 1, 0, 0};
}

__device__ __forceinline__ RunCursor linear_run(const SeqArgs &a) {
    if (a.queue)
        return RunCursor{0, 0, a.chunk, a.chunk, 0, 0, 0, 1};
    return RunCursor{(uint64_t)blockIdx.x * a.chunk, a.n_tiles, 0, a.chunk, gridDim.x, 0, 0, 0};
}

// Next tile of the walk, or false at its end.
__device__ __forceinline__ bool run_next(const SeqArgs &a, RunCursor &rc, uint64_t *tile) {
    if (a.queue) {
        __shared__ uint32_t claimed;
        for (;;) {
            if (rc.gi < rc.G && rc.c + rc.gi < rc.end) {
                const uint64_t j = rc.c + rc.gi++;
                *tile = rc.ordered ? (uint64_t)a.tile_order[j] : j;
                return true;
            }
            if (!rc.qleft)
                return false;
            // claim the next chunk of share qx
            const uint64_t lo = rc.ordered ? a.xcd_start[rc.qx] : 0;
            const uint64_t hi = rc.ordered ? a.xcd_start[rc.qx + 1] : a.n_tiles;
            __syncthreads();  // every thread has read the last claim
            if (threadIdx.x == 0)
                claimed = atomicAdd(&a.queue[rc.qx], rc.G);
            __syncthreads();
            const uint64_t c = lo + claimed;
            if (c < hi) {
                rc.c = c;
                rc.end = hi;
                rc.gi = 0;
            } else {  // share exhausted: the next one
                rc.qx = rc.ordered ? (rc.qx + 1) % NXCD : 0;
                --rc.qleft;
                rc.gi = rc.G;
            }
        }
    }
    while (rc.c < rc.end) {
        if (rc.gi < rc.G && rc.c + rc.gi < rc.end) {
            const uint64_t j = rc.c + rc.gi++;
            *tile = rc.ordered ? (uint64_t)a.tile_order[j] : j;
            return true;
        }
        rc.c += (uint64_t)rc.step * rc.G;
        rc.gi = 0;
    }
    return false;
}

// Wave-wide ballot as a 64-bit mask (wave64).
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// A per-set counter summed over the tiles a persistent workgroup walks.  Each
// thread keeps its part for the current set in a register; when the tile's
// set changes, and at the end, the workgroup adds the parts in LDS and issues
// one device atomic.  (Atomics on one address from every XCD serialise far
// from the CUs, so one per tile or per thread would dominate the kernel.)
// Every call must be reached by the whole workgroup with the same `set`.
struct SetSum {
    uint32_t set;
    unsigned long long v;
};

__device__ __forceinline__ SetSum setsum_begin() { return SetSum{~0u, 0ull}; }

__device__ __forceinline__ void setsum_flush(SetSum &s, unsigned long long *lds,
                                             unsigned long long *counter_of_set0,
                                             uint32_t stride_words) {
    if (s.set == ~0u)
        return;
    if (threadIdx.x == 0)
        *lds = 0;
    __syncthreads();
    if (s.v)
        atomicAdd(lds, s.v);
    __syncthreads();
    if (threadIdx.x == 0 && *lds)
        atomicAdd(counter_of_set0 + (uint64_t)s.set * stride_words, *lds);
    s.v = 0;
}

// Switch the sum to `set` (flushing the previous set's part when it differs).
__device__ __forceinline__ void setsum_switch(SetSum &s, uint32_t set, unsigned long long *lds,
                                              unsigned long long *counter_of_set0,
                                              uint32_t stride_words) {
    if (set != s.set) {
        setsum_flush(s, lds, counter_of_set0, stride_words);
        s.set = set;
    }
}

constexpr uint32_t SETCNT_STRIDE = sizeof(SetCounters) / sizeof(unsigned long long);

// ------------------------------------------------ binned schedules (LDS sort)

constexpr uint64_t BIN_NONE = ~0ull;  // no item (real items never have all bits set)

// Exclusive scan of the N counters cnt[] into start[] by NT threads
// (N / NT consecutive counters per thread, or one for the first N threads
// when N < NT); the total goes to *total.  Called by the whole workgroup;
// ends synchronised.
template <uint32_t N, uint32_t NT>
__device__ __forceinline__ void lds_scan(const uint32_t *cnt, uint32_t *start, uint32_t *wtot,
                                         uint32_t *total) {
    static_assert(NT % 64 == 0 && (N >= NT ? N % NT == 0 : NT % N == 0), "scan shape");
    constexpr uint32_t E = N >= NT ? N / NT : 1;
    const uint32_t t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t c[E], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < E; ++q) {
        c[q] = t * E + q < N ? cnt[t * E + q] : 0;
        sum += c[q];
    }
    uint32_t x = sum;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    if (lane == 63)
        wtot[wave] = x;
    __syncthreads();
    uint32_t before = 0;
    for (uint32_t q = 0; q < wave; ++q)
        before += wtot[q];
    uint32_t e = before + x - sum;
#pragma unroll
    for (uint32_t q = 0; q < E; ++q) {
        if (t * E + q < N)
            start[t * E + q] = e;
        e += c[q];
    }
    if (t == NT - 1)
        *total = e;
    __syncthreads();
}

// Exclusive scan of n counts into n + 1 offsets (the last one the total), by
// one workgroup: rounds of 4 counts per thread, a wave scan of the thread
// sums, then the wave totals.
__device__ __forceinline__ void bin_offsets_scan(const uint32_t *counts, uint64_t n,
                                                 uint64_t *offsets) {
    constexpr uint32_t WAVES = BIN_SCAN_BLOCK / 64;
    __shared__ uint64_t wsum[WAVES];
    __shared__ uint64_t carry_s;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0)
        carry_s = 0;
    for (uint64_t base = 0; base < n; base += 4ull * BIN_SCAN_BLOCK) {
        const uint64_t i0 = base + 4ull * threadIdx.x;
        uint64_t v[4], t = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            v[q] = i0 + q < n ? counts[i0 + q] : 0;
            t += v[q];
        }
        uint64_t x = t;  // inclusive scan of the thread sums within the wave
#pragma unroll
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint64_t y = (uint64_t)__shfl_up((long long)x, d, 64);
            if (lane >= d)
                x += y;
        }
        __syncthreads();  // carry_s of the last round is in place
        if (lane == 63)
            wsum[wave] = x;
        __syncthreads();
        uint64_t before = carry_s;
        for (uint32_t q = 0; q < wave; ++q)
            before += wsum[q];
        uint64_t c = before + x - t;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (i0 + q < n)
                offsets[i0 + q] = c;
            c += v[q];
        }
        __syncthreads();
        if (threadIdx.x == BIN_SCAN_BLOCK - 1)
            carry_s = c;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        offsets[n] = carry_s;
}

// Write a batch of items, PER per thread (BIN_NONE: none), to their bins'
// cursors in out: the batch sorted by bin (bin_of(item) < NB) in LDS
// (counting sort), then the sorted items written in order, so that a bin's
// items of the batch go out as one contiguous run.  A 32-bit out keeps the
// low 32 bits of each item.  cnt[] must be zero on
// entry and is zero again on return; cursor[] advances by each bin's count.
// Whole workgroup; ends synchronised.
template <uint32_t NB, uint32_t NT, uint32_t PER, class BinOf, class Out>
__device__ __forceinline__ void sorted_write_by(const uint64_t (&v)[PER], BinOf bin_of,
                                                uint32_t *cnt, uint32_t *start, uint32_t *wtot,
                                                uint32_t *total, uint64_t *srt, uint64_t *cursor,
                                                Out *out) {
    uint32_t rk[PER];
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q)
        rk[q] = v[q] != BIN_NONE ? atomicAdd(&cnt[bin_of(v[q])], 1u) : 0;
    __syncthreads();
    lds_scan<NB, NT>(cnt, start, wtot, total);
#pragma unroll
    for (uint32_t q = 0; q < PER; ++q)
        if (v[q] != BIN_NONE)
            srt[start[bin_of(v[q])] + rk[q]] = v[q];
    __syncthreads();
    const uint32_t n = *total;
    for (uint32_t i = threadIdx.x; i < n; i += NT) {
        const uint64_t it = srt[i];
        const uint32_t bn = bin_of(it);
        out[cursor[bn] + (i - start[bn])] = (Out)it;
    }
    __syncthreads();
    for (uint32_t bn = threadIdx.x; bn < NB; bn += NT) {
        cursor[bn] += cnt[bn];
        cnt[bn] = 0;
    }
    __syncthreads();
}


}  // namespace tp
