// Ordered compaction of the junction bitmap and the compacted edges
// (Reduction section: the vertices of the compacted graph are the k-mers at
// junction positions, and every two consecutive junction positions of one
// string give an edge), for gfx950.
//
//   k_block_counts  popcount of SCAN_WORDS bitmap words per workgroup
//   k_scan_blocks   exclusive scan of the workgroup counts (one workgroup)
//   k_emit          per workgroup: wave shuffle scan + LDS scan of word
//                   popcounts, then every set bit writes its junction in
//                   global order (genome coordinate, normalised k-mer,
//                   strand) and its share of the edges: junction n of string
//                   s starts edge n - s unless it is the string's last k-mer,
//                   and ends edge n - 1 - s unless it is the string's first
//                   (both are always junctions, so every string of c
//                   junctions owns c - 1 consecutive edges, and the strings
//                   before s own exactly s more junctions than edges)
//   k_joff          per genome: its first junction index, the number of set
//                   bitmap bits before its first base (a rank query)
#include "device.hpp"

namespace tp {

// Exclusive scan of one value per thread over a BLOCK-thread workgroup.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total,
                                                         uint32_t *wsum) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d)
            x += y;
    }
    if (lane == 63)
        wsum[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (uint32_t i = 0; i < BLOCK / 64; ++i) {
        pre += i < wid ? wsum[i] : 0;
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(BLOCK) void k_block_counts(const uint64_t *bits, uint64_t nwords,
                                                        uint32_t *blockcnt) {
    __shared__ uint32_t wsum[BLOCK / 64];
    uint32_t c = 0;
    const uint64_t w0 = (uint64_t)blockIdx.x * SCAN_WORDS;
    for (uint32_t i = 0; i < SCAN_WORDS / BLOCK; ++i) {
        const uint64_t wi = w0 + i * BLOCK + threadIdx.x;
        if (wi < nwords)
            c += (uint32_t)__popcll(bits[wi]);
    }
    uint32_t tot;
    block_exclusive_scan(c, &tot, wsum);
    if (threadIdx.x == 0)
        blockcnt[blockIdx.x] = tot;
}

__global__ __launch_bounds__(BLOCK) void k_scan_blocks(const uint32_t *blockcnt, uint32_t nblocks,
                                                       uint64_t *blockoff) {
    __shared__ uint32_t wsum[BLOCK / 64];
    uint64_t running = 0;
    for (uint32_t b0 = 0; b0 < nblocks; b0 += BLOCK) {
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nblocks ? blockcnt[b] : 0;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, &tot, wsum);
        if (b < nblocks)
            blockoff[b] = running + ex;
        running += tot;
    }
    if (threadIdx.x == 0)
        blockoff[nblocks] = running;
}

// Junctions in global order.  Each of SCAN_WORDS / BLOCK rounds scans BLOCK
// bitmap words (one per thread): each thread writes the in-round positions of
// its word's set bits into an LDS index at its scanned offset (one short
// store per junction, no search), then thread t writes junctions t, t +
// BLOCK, ... of the round, so consecutive threads write consecutive outputs
// (coalesced) whatever the junction density.
template <class T>
__global__ __launch_bounds__(BLOCK) void k_emit(SeqArgs a, const uint64_t *bits, uint64_t nwords,
                                                const uint64_t *blockoff, OutArgs o, uint64_t nj,
                                                uint64_t ne) {
    // the round's k-mers: its BLOCK * 64 positions, plus the longest window
    constexpr uint32_t EMIT_WORDS = BLOCK * 64 / 32 + 5;
    __shared__ uint32_t wsum[BLOCK / 64];
    __shared__ uint16_t jpos[BLOCK * 64];  // junction j of the round: word << 6 | bit
    __shared__ uint64_t gw[EMIT_WORDS];
    static_assert(BLOCK * 64 <= 65536, "in-round positions fit 16 bits");
    const uint32_t k = a.k;
    const bool single = a.single != 0;
    uint64_t running = blockoff[blockIdx.x];
    const uint64_t w0 = (uint64_t)blockIdx.x * SCAN_WORDS;
    uint32_t si = a.n_strings;
    uint64_t gs = ~0ull, ge = 0;
    for (uint32_t i = 0; i < SCAN_WORDS / BLOCK; ++i) {
        const uint64_t wbase = w0 + (uint64_t)i * BLOCK;
        const uint64_t wi = wbase + threadIdx.x;
        const uint64_t word = wi < nwords ? bits[wi] : 0;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan((uint32_t)__popcll(word), &tot, wsum);
        {
            uint32_t at = ex;
            for (uint64_t x = word; x; x &= x - 1)
                jpos[at++] = (uint16_t)(threadIdx.x << 6 | (uint32_t)__builtin_ctzll(x));
        }
        const uint64_t pbase = wbase * 64;
        if (tot) {
            for (uint32_t u = threadIdx.x; u < EMIT_WORDS; u += BLOCK) {
                const uint64_t q = pbase / 32 + u;
                gw[u] = q < a.seq_words ? a.seq[q] : 0ull;
            }
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < tot; j += BLOCK) {
            const uint64_t n = running + j;
            if (n >= nj)
                break;
            const uint64_t p = pbase + jpos[j];
            if (p < gs || p >= ge) {
                const TileInfo ti = a.tiles[p / TILE];
                si = find_string(a.strings, ti.str_lo, ti.str_hi, p);
                if (si == ti.str_hi)
                    si = 0;  // unreachable: junction bits lie inside strings
                gs = a.strings[si].gstart;
                ge = a.strings[si].gend;
            }
            const uint32_t g = a.strings[si].genome;
            const Strands<T> st = strands(KT<T>::window(gw, (uint32_t)(p - pbase), k), k);
            const bool fwd_is_norm = single || st.fwd <= st.rc;
            const T v = fwd_is_norm ? st.fwd : st.rc;
            const uint64_t gp = p - o.gbase[g];
            o.pos[n] = gp;
#pragma unroll
            for (uint32_t wd = 0; wd < (uint32_t)KT<T>::W; ++wd)
                o.vertex[n * KT<T>::W + wd] = KT<T>::word(v, wd);
            o.strand[n] = fwd_is_norm ? 0 : 1;
            // edge words: (genome | flags << 32, from, to), 24 bytes each
            uint64_t *ew = (uint64_t *)o.edges;
            // (the index checks only guard the buffer; they hold by construction)
            if (p + k != ge && n >= si && n - si < ne) {  // starts edge n - si
                ew[3 * (n - si)] = g;
                ew[3 * (n - si) + 1] = gp;
            }
            if (p != gs && n > si && n - 1 - si < ne)  // ends edge n - 1 - si
                ew[3 * (n - 1 - si) + 2] = gp;
        }
        running += tot;
        __syncthreads();
    }
}

// joff[g] = set bits before genome g's first base (g < n_genomes), one
// workgroup per genome: the scanned count of the bits' compaction block plus
// the popcounts of that block's words before the genome's first word.
// Genomes start on tile boundaries, hence on word boundaries.
__global__ __launch_bounds__(BLOCK) void k_joff(const uint64_t *bits, uint64_t nwords,
                                                const uint64_t *blockoff, OutArgs o) {
    __shared__ uint32_t wsum[BLOCK / 64];
    const uint64_t nj = blockoff[(nwords + SCAN_WORDS - 1) / SCAN_WORDS];  // all set bits
    const uint32_t g = blockIdx.x;
    const uint64_t w = o.gbase[g] / 64;
    const uint64_t b = w / SCAN_WORDS;
    uint32_t c = 0;
    for (uint64_t i = b * SCAN_WORDS + threadIdx.x; i < w && i < nwords; i += BLOCK)
        c += (uint32_t)__popcll(bits[i]);
    uint32_t tot;
    block_exclusive_scan(c, &tot, wsum);
    if (threadIdx.x == 0)
        o.joff[g] = w >= nwords ? nj : blockoff[b] + tot;
    if (threadIdx.x == 0 && g + 1 == o.n_genomes)
        o.joff[o.n_genomes] = nj;
}

hipError_t launch_compact(int W, const SeqArgs &a, const uint64_t *jbits, uint64_t nwords,
                          uint32_t *blockcnt, uint64_t *blockoff, const OutArgs &o,
                          uint64_t n_junctions, hipStream_t s) {
    if (n_junctions == 0)
        return launch_fill_u64(o.joff, (uint64_t)o.n_genomes + 1, 0, s);
    const uint32_t nblocks = (uint32_t)((nwords + SCAN_WORDS - 1) / SCAN_WORDS);
    const uint64_t ne = n_junctions >= a.n_strings ? n_junctions - a.n_strings : 0;
    hipLaunchKernelGGL(k_block_counts, dim3(nblocks), dim3(BLOCK), 0, s, jbits, nwords, blockcnt);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(BLOCK), 0, s, blockcnt, nblocks, blockoff);
    (void)by_width(W, [&](auto tag) {
        hipLaunchKernelGGL(k_emit<decltype(tag)>, dim3(nblocks), dim3(BLOCK), 0, s, a, jbits,
                           nwords, blockoff, o, n_junctions, ne);
        return hipSuccess;
    });
    if (o.n_genomes)
        hipLaunchKernelGGL(k_joff, dim3(o.n_genomes), dim3(BLOCK), 0, s, jbits, nwords, blockoff,
                           o);
    return hipGetLastError();
}

hipError_t launch_compact_bound(int W, const SeqArgs &a, const uint64_t *jbits, uint64_t nwords,
                                uint32_t *blockcnt, uint64_t *blockoff, const OutArgs &o,
                                uint64_t max_j, uint64_t max_e, hipStream_t s) {
    if (nwords == 0)
        return launch_fill_u64(o.joff, (uint64_t)o.n_genomes + 1, 0, s);
    const uint32_t nblocks = (uint32_t)((nwords + SCAN_WORDS - 1) / SCAN_WORDS);
    hipLaunchKernelGGL(k_block_counts, dim3(nblocks), dim3(BLOCK), 0, s, jbits, nwords, blockcnt);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(BLOCK), 0, s, blockcnt, nblocks, blockoff);
    (void)by_width(W, [&](auto tag) {
        hipLaunchKernelGGL(k_emit<decltype(tag)>, dim3(nblocks), dim3(BLOCK), 0, s, a, jbits,
                           nwords, blockoff, o, max_j, max_e);
        return hipSuccess;
    });
    if (o.n_genomes)
        hipLaunchKernelGGL(k_joff, dim3(o.n_genomes), dim3(BLOCK), 0, s, jbits, nwords, blockoff,
                           o);
    return hipGetLastError();
}

// Counts of a caller-memory run: per-set sums, the junction total from the
// compaction scan, edges = junctions - strings (every string of c junctions
// has c - 1 edges), and a status word.
__global__ __launch_bounds__(BLOCK) void k_ws_finalize(FinalizeArgs f) {
    __shared__ unsigned long long part[5][BLOCK];
    unsigned long long c[5] = {0, 0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < f.n_sets; i += BLOCK) {
        const SetCounters &sc = f.set_cnt[i];
        c[0] += sc.candidates;
        c[1] += sc.bloom_popcount;
        c[2] += sc.table_keys;
        c[3] += sc.overflow ? 1ull : 0ull;
        c[4] += sc.junctions;
    }
    for (int q = 0; q < 5; ++q)
        part[q][threadIdx.x] = c[q];
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    for (uint32_t t = 1; t < BLOCK; ++t)
        for (int q = 0; q < 5; ++q)
            c[q] += part[q][t];
    const uint64_t nj = f.nblocks ? f.blockoff[f.nblocks] : 0;
    unsigned long long status = 0;
    if (f.pass2 && c[3])
        status |= 1;  // a table overflowed: its set's tiles were skipped
    if (nj > f.max_j)
        status |= 2;
    if (f.cnt->missing || (nj && nj < f.n_strings))
        status |= 4;
    f.out[0] = status;
    f.out[1] = f.positions;
    f.out[2] = c[0];
    f.out[3] = nj;
    f.out[4] = nj >= f.n_strings ? nj - f.n_strings : 0;
    f.out[5] = c[2];
    f.out[6] = c[1];
    for (int q = 7; q < 16; ++q)
        f.out[q] = 0;
}

hipError_t launch_ws_finalize(const FinalizeArgs &f, hipStream_t s) {
    hipLaunchKernelGGL(k_ws_finalize, dim3(1), dim3(BLOCK), 0, s, f);
    return hipGetLastError();
}

}  // namespace tp
