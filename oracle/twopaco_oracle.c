/*
 * TwoPaCo junction-finding oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation written from the paper
 * (Minkin, Pham & Medvedev, "TwoPaCo: An efficient algorithm to build the
 * compacted de Bruijn graph from many complete genomes", arXiv 1602.05856).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file.  It shares no code, header or constant table
 * with the GPU library, and the GPU library never loads it.
 *
 * Functions
 *   or_bruteforce    J(S,k) straight from the definitions of the
 *                    Preliminaries section (bifurcation, sentinel, junction)
 *                    applied to the comprehensive graph G(S) u G(S-bar): the
 *                    reverse-complement strings are built explicitly and no
 *                    k-mer is ever normalised.
 *   or_twopass       Algorithm 2 (Filter-Junctions-Two-Pass) with a single
 *                    round (Algorithm 3 with l = 1), i.e. Algorithm 1
 *                    (Filter-Junctions) run first with a Bloom filter and then
 *                    with an exact set, on normalised k-mers as the
 *                    reverse-complement paragraph of the Single Round section
 *                    prescribes.
 *   or_vertex        normalised k-mer and strand of given positions.
 *   or_edges         compacted edges: consecutive junctions of one string
 *                    (Reduction section, Observation 1).
 *   or_vertex_masks  in- and out-edges and sentinel status of given vertices
 *                    of the comprehensive graph, by the definitions, in one
 *                    streaming pass (for inputs too large for brute force);
 *                    or_sample_status the junction status of sampled
 *                    positions from them.  Both also take packed input.
 *   or_rounds        Algorithm 3 with l >= 1 rounds: k-mers split into l
 *                    classes by the greedy partition heuristic of the Multiple
 *                    Rounds section, Algorithm 2 run once per class, marks
 *                    united.
 *
 * Filter variants (the paper fixes neither the hash family nor the layout of
 * its Bloom filter; both variants below are Bloom filters over the edge set,
 * with no false negatives):
 *   standard  h bit positions anywhere in the b bits (double hashing);
 *   blocked   (flag OR_BLOCKED) all h bits of an edge in one 64-bit block,
 *             the block chosen by the edge's middle (k-1)-mer (see
 *             blocked_indices), so the edges around one k-mer share blocks.
 *
 * Parity status
 *   Junction positions, vertices, edges: pinned (brute force vs the two-pass
 *   run, worked example of Fig. 1, closed forms, invariants).
 *   Bloom filter bits and the pass-1 candidate set: they depend on the hash
 *   family, which the paper leaves open (Theoretical Analysis section only
 *   says "sliding window hash functions").  They are pinned only by
 *   structural and statistical properties (no false negatives, fill ratio and
 *   false-positive rate of the Theoretical Analysis section, candidates equal
 *   junctions when the filter has no collisions); their exact bit values are
 *   parity unpinned.
 *
 * Conventions (readings of the paper where it is silent)
 *   codes      A=0 C=1 G=2 T=3; any code > 3 is N.  A string of S is a maximal
 *              N-free run ("contig") of a genome.
 *   positions  0-based k-mer start, genome coordinates.
 *   value      val(x) = sum_t x[t] * 4^(L-1-t) (first base most significant),
 *              so unsigned order is lexicographic order with A<C<G<T.
 *   normalised min(val(x), val(rc(x))); with TP single-strand flag it is val(x).
 *   hash       Bloom bit t of a (k+1)-mer e:  (H1 + t*H2) mod 2^64 mod b with
 *              H1 = mix64(fold(e) ^ S1), H2 = mix64(fold(e) ^ S2) | 1,
 *              fold(e) = e for k <= 31; else, over the W words of e (W = 2
 *              for k <= 63, 4 for k <= 127), f = top word, then
 *              f = mix64(f ^ S0) ^ word for each lower word; mix64 the
 *              SplitMix64 finaliser (Steele, Lea & Flood, OOPSLA 2014).
 *   k          1 <= k <= 127 (values of up to 128 bases in four words).
 *              Double hashing after Kirsch & Mitzenmacher (ESA 2006).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* A value of up to 128 bases (2 bits each): four 64-bit words, w[0] least
 * significant. */
typedef struct {
    uint64_t w[4];
} kv;

static kv kv_zero(void)
{
    kv v = {{0, 0, 0, 0}};
    return v;
}

/* v = 4 v + c */
static void kv_push(kv *v, uint8_t c)
{
    v->w[3] = (v->w[3] << 2) | (v->w[2] >> 62);
    v->w[2] = (v->w[2] << 2) | (v->w[1] >> 62);
    v->w[1] = (v->w[1] << 2) | (v->w[0] >> 62);
    v->w[0] = (v->w[0] << 2) | c;
}

/* Unsigned comparison: -1, 0, 1. */
static int kv_cmp(kv a, kv b)
{
    for (int i = 3; i >= 0; --i)
        if (a.w[i] != b.w[i])
            return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

static kv kv_words(const uint64_t *w)
{
    kv v = {{w[0], w[1], w[2], w[3]}};
    return v;
}

#define OR_SINGLE_STRAND 1u
#define OR_BLOCKED 4u

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2 };

/* ---------------------------------------------------------------- hash spec */

static const uint64_t OR_S0 = 0x243F6A8885A308D3ull; /* hex digits of pi */
static const uint64_t OR_S1 = 0x13198A2E03707344ull;
static const uint64_t OR_S2 = 0xA4093822299F31D0ull;

/* SplitMix64 output function (Steele, Lea & Flood 2014): two
 * xorshift-multiply rounds and a final xorshift. */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* One 64-bit word from a value held in W words (W = 1 for k <= 31, 2 for
 * k <= 63, 4 for k <= 127): the top word, then for each lower word
 * f = mix64(f ^ S0) ^ word. */
static uint64_t fold(kv x, uint32_t k)
{
    const int W = k <= 31 ? 1 : (k <= 63 ? 2 : 4);
    uint64_t f = x.w[W - 1];
    for (int i = W - 2; i >= 0; --i)
        f = or_mix64(f ^ OR_S0) ^ x.w[i];
    return f;
}

/* The h bit indices of (k+1)-mer value e in a Bloom filter of b bits. */
static void bloom_indices(kv e, uint32_t k, uint64_t b, uint32_t h, uint64_t *idx)
{
    uint64_t f = fold(e, k);
    uint64_t h1 = or_mix64(f ^ OR_S1);
    uint64_t h2 = or_mix64(f ^ OR_S2) | 1ull;
    for (uint32_t t = 0; t < h; ++t)
        idx[t] = (h1 + (uint64_t)t * h2) & (b - 1);
}

/* Exported so the tests can check the spec on fixed vectors (value given
 * as four words, least significant first). */
void or_bloom_indices(const uint64_t *words, uint32_t k, uint64_t b, uint32_t h, uint64_t *idx)
{
    bloom_indices(kv_words(words), k, b, h, idx);
}

/* ------------------------------------------------------------ strings, k-mers */

typedef struct {
    const uint8_t *codes; /* base codes, > 3 means N */
    uint64_t len;
} or_genome;

typedef struct {
    uint32_t genome;
    uint64_t start; /* genome coordinate of the first base */
    uint64_t len;
} contig_t;

/* val of the L-mer s[i..i+L-1], first base most significant. */
static kv val(const uint8_t *s, uint64_t i, uint32_t L)
{
    kv v = kv_zero();
    for (uint32_t t = 0; t < L; ++t)
        kv_push(&v, s[i + t]);
    return v;
}

/* val of the reverse complement of s[i..i+L-1]. */
static kv rcval(const uint8_t *s, uint64_t i, uint32_t L)
{
    kv v = kv_zero();
    for (uint32_t t = 0; t < L; ++t)
        kv_push(&v, (uint8_t)(3 - s[i + L - 1 - t]));
    return v;
}

/* Normalised form: the lexicographically smaller of x and its reverse
 * complement (reverse-complement paragraph, Single Round section). */
static kv norm(const uint8_t *s, uint64_t i, uint32_t L, uint32_t flags)
{
    kv f = val(s, i, L);
    if (flags & OR_SINGLE_STRAND)
        return f;
    kv r = rcval(s, i, L);
    return kv_cmp(f, r) < 0 ? f : r;
}

/* Blocked-filter bit indices of the (k+1)-mer e[0..k] = x.m.y (x = e[0],
 * y = e[k], m the k-1 bases between).  The edge is written in the
 * orientation in which its middle is normalised: (p, q) = (x, y) when
 * val(m) < val(rc(m)), (3-y, 3-x) when val(m) > val(rc(m)); a palindromic
 * middle takes the orientation of the normalised edge.  With mu the
 * normalised middle, f = fold(mu):
 *   block = mix64(f ^ S1) mod (b/64), G = mix64(f ^ S2),
 *   a = G & 63, d = ((G >> 6) & 63) | 1, j = 4p + q,
 *   bit t (t < h) = 64*block + ((a + (j*h + t)*d) mod 64).
 * e and its reverse complement get the same bits.  For h <= 4 the 16 edges
 * with one middle use disjoint bits of their block. */
static void blocked_indices(const uint8_t *e, uint32_t k, uint64_t b, uint32_t h, uint32_t flags,
                            uint64_t *idx)
{
    kv mf = val(e, 1, k - 1);
    kv mr = (flags & OR_SINGLE_STRAND) ? mf : rcval(e, 1, k - 1);
    uint8_t x = e[0], y = e[k], p, q;
    kv mu;
    const int c = kv_cmp(mf, mr);
    if ((flags & OR_SINGLE_STRAND) || c < 0) {
        mu = mf;
        p = x;
        q = y;
    } else if (c > 0) {
        mu = mr;
        p = (uint8_t)(3 - y);
        q = (uint8_t)(3 - x);
    } else {
        mu = mf;
        if (kv_cmp(val(e, 0, k + 1), rcval(e, 0, k + 1)) <= 0) {
            p = x;
            q = y;
        } else {
            p = (uint8_t)(3 - y);
            q = (uint8_t)(3 - x);
        }
    }
    uint64_t f = fold(mu, k);
    uint64_t block = or_mix64(f ^ OR_S1) & (b / 64 - 1);
    uint64_t g = or_mix64(f ^ OR_S2);
    uint64_t a = g & 63, d = ((g >> 6) & 63) | 1, j = 4u * p + q;
    for (uint32_t t = 0; t < h; ++t)
        idx[t] = 64 * block + ((a + (j * h + t) * d) & 63);
}

/* Exported for the tests: blocked-filter indices of the (k+1)-mer given as
 * base codes. */
void or_blocked_indices(const uint8_t *e, uint32_t k, uint64_t b, uint32_t h, uint32_t flags,
                        uint64_t *idx)
{
    blocked_indices(e, k, b, h, flags, idx);
}

/* Split every genome into maximal N-free runs. */
static contig_t *make_contigs(const or_genome *g, uint32_t n, uint64_t *n_out)
{
    uint64_t cap = 16, cnt = 0;
    contig_t *c = (contig_t *)malloc(cap * sizeof(contig_t));
    if (!c)
        return NULL;
    for (uint32_t gi = 0; gi < n; ++gi) {
        uint64_t j = 0;
        while (j < g[gi].len) {
            if (g[gi].codes[j] > 3) {
                ++j;
                continue;
            }
            uint64_t s = j;
            while (j < g[gi].len && g[gi].codes[j] <= 3)
                ++j;
            if (cnt == cap) {
                cap *= 2;
                contig_t *nc = (contig_t *)realloc(c, cap * sizeof(contig_t));
                if (!nc) {
                    free(c);
                    return NULL;
                }
                c = nc;
            }
            c[cnt].genome = gi;
            c[cnt].start = s;
            c[cnt].len = j - s;
            ++cnt;
        }
    }
    *n_out = cnt;
    return c;
}

/* ------------------------------------------------------- sorted value sets */

static int cmp_kv(const void *a, const void *b)
{
    return kv_cmp(*(const kv *)a, *(const kv *)b);
}

typedef struct {
    kv *v;
    uint64_t n, cap;
} vset;

static int vset_push(vset *s, kv x)
{
    if (s->n == s->cap) {
        uint64_t nc = s->cap ? s->cap * 2 : 1024;
        kv *nv = (kv *)realloc(s->v, nc * sizeof(kv));
        if (!nv)
            return OR_ENOMEM;
        s->v = nv;
        s->cap = nc;
    }
    s->v[s->n++] = x;
    return OR_OK;
}

/* Sort and drop duplicates. */
static void vset_finish(vset *s)
{
    if (s->n == 0)
        return;
    qsort(s->v, s->n, sizeof(kv), cmp_kv);
    uint64_t w = 1;
    for (uint64_t r = 1; r < s->n; ++r)
        if (kv_cmp(s->v[r], s->v[w - 1]) != 0)
            s->v[w++] = s->v[r];
    s->n = w;
}

static int vset_has(const vset *s, kv x)
{
    uint64_t lo = 0, hi = s->n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (kv_cmp(s->v[mid], x) < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo < s->n && kv_cmp(s->v[lo], x) == 0;
}

/* ------------------------------------------------ the edge-set abstraction E */

/* Algorithm 1 takes an empty set data structure E with insert and member.
 * Two implementations: a Bloom filter (first pass) and an exact set (second
 * pass).  The exact set collects inserts and is sorted before the queries,
 * which is legal because the two loops of Algorithm 1 are separated. */
typedef struct {
    int is_bloom;
    uint32_t k, h, flags;
    uint64_t b;
    uint32_t *words; /* Bloom: bit i is bit (i & 31) of words[i >> 5] */
    vset exact;
} edge_set;

/* Filter bit indices of the edge given as k+1 base codes. */
static void filter_indices(const edge_set *E, const uint8_t *e, uint64_t *idx)
{
    if (E->flags & OR_BLOCKED)
        blocked_indices(e, E->k, E->b, E->h, E->flags, idx);
    else
        bloom_indices(norm(e, 0, E->k + 1, E->flags), E->k, E->b, E->h, idx);
}

static int eset_insert(edge_set *E, const uint8_t *e)
{
    if (E->is_bloom) {
        uint64_t idx[64];
        filter_indices(E, e, idx);
        for (uint32_t t = 0; t < E->h; ++t)
            E->words[idx[t] >> 5] |= 1u << (idx[t] & 31);
        return OR_OK;
    }
    return vset_push(&E->exact, norm(e, 0, E->k + 1, E->flags));
}

static void eset_seal(edge_set *E)
{
    if (!E->is_bloom)
        vset_finish(&E->exact);
}

static int eset_member(const edge_set *E, const uint8_t *e)
{
    if (E->is_bloom) {
        uint64_t idx[64];
        filter_indices(E, e, idx);
        for (uint32_t t = 0; t < E->h; ++t)
            if (!(E->words[idx[t] >> 5] & (1u << (idx[t] & 31))))
                return 0;
        return 1;
    }
    return vset_has(&E->exact, norm(e, 0, E->k + 1, E->flags));
}

/* ------------------------------------------------------ Algorithm 1 */

/* Normalised sentinel set: first and last k-mer of every string.  The first
 * k-mer of a reverse complement is the reverse complement of the last k-mer,
 * so normalising covers both strands. */
static int make_sentinels(const or_genome *g, const contig_t *c, uint64_t nc, uint32_t k,
                          uint32_t flags, vset *sent)
{
    for (uint64_t i = 0; i < nc; ++i) {
        if (c[i].len < k)
            continue;
        const uint8_t *s = g[c[i].genome].codes + c[i].start;
        if (vset_push(sent, norm(s, 0, k, flags)) || vset_push(sent, norm(s, c[i].len - k, k, flags)))
            return OR_ENOMEM;
    }
    vset_finish(sent);
    return OR_OK;
}

/* In- and out-degree of the vertex v (the k bases at v) in the graph whose
 * edge set is E: the number of bases c with c.v in E, and the number with
 * v.c in E (Preliminaries section: a bifurcation has more than one of
 * either). */
static void degrees(const edge_set *E, const uint8_t *v, uint32_t k, int *in, int *out)
{
    uint8_t e[130];
    *in = *out = 0;
    for (uint8_t c = 0; c < 4; ++c) {
        memcpy(e, v, k); /* v followed by c */
        e[k] = c;
        *out += eset_member(E, e);
        e[0] = c; /* c followed by v */
        memcpy(e + 1, v, k);
        *in += eset_member(E, e);
    }
}

/* Filter-Junctions (Algorithm 1) on the candidate set C, given as marks[g][pos]
 * (one byte per genome position), updated in place.
 *
 * Build E: the text of the Single Round section puts into E every (k+1)-mer
 * of a string whose first or second k-mer is in C.  (For a string of exactly
 * k+1 bases this inserts its lone edge; both of its k-mers are sentinels, so
 * the junctions do not depend on it.)
 *
 * Filter C: a marked position keeps its mark exactly when its k-mer is a
 * junction of the graph that E describes -- a sentinel (the normalised first
 * or last k-mer of some string), or a vertex with more than one in-edge or
 * more than one out-edge in E.  Every edge of a marked position's own
 * predecessor and successor went into E, so with E exact this leaves J(S,k)
 * among the marks, and with a filter without false negatives a superset of
 * it. */
static int filter_junctions(const or_genome *g, const contig_t *c, uint64_t nc, uint32_t k,
                            uint32_t flags, const vset *sent, edge_set *E, uint8_t **marks)
{
    for (uint64_t ci = 0; ci < nc; ++ci) {
        const uint8_t *s = g[c[ci].genome].codes + c[ci].start;
        const uint8_t *C = marks[c[ci].genome] + c[ci].start;
        for (uint64_t j = 0; j + k + 1 <= c[ci].len; ++j)
            if (C[j] || C[j + 1])
                if (eset_insert(E, s + j))
                    return OR_ENOMEM;
    }
    eset_seal(E);
    for (uint64_t ci = 0; ci < nc; ++ci) {
        const uint8_t *s = g[c[ci].genome].codes + c[ci].start;
        uint8_t *C = marks[c[ci].genome] + c[ci].start;
        for (uint64_t i = 0; i + k <= c[ci].len; ++i) {
            if (!C[i] || vset_has(sent, norm(s, i, k, flags)))
                continue;
            int in, out;
            degrees(E, s + i, k, &in, &out);
            C[i] = in > 1 || out > 1;
        }
    }
    return OR_OK;
}

typedef struct {
    uint64_t positions;      /* k-mer positions over all strings       */
    uint64_t marks_pass1;    /* marks left after the first pass        */
    uint64_t marks_pass2;    /* marks left after the second pass (= |J|) */
    uint64_t bloom_popcount; /* set bits of the filter                 */
    uint64_t exact_edges;    /* distinct (k+1)-mers in the exact set   */
    uint64_t distinct_edges; /* distinct normalised (k+1)-mers, all    */
} or_stats;

static int check_args(uint32_t k, uint64_t b, uint32_t h, uint32_t flags)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    if (b < ((flags & OR_BLOCKED) ? 64u : 32u) || (b & (b - 1)))
        return OR_EINVAL;
    if (h < 1 || h > 64)
        return OR_EINVAL;
    return OR_OK;
}

/* Mark every k-mer start of every string (C_in with all positions marked). */
static void mark_all(const contig_t *c, uint64_t nc, uint32_t k, uint8_t **marks, uint64_t *npos)
{
    uint64_t p = 0;
    for (uint64_t ci = 0; ci < nc; ++ci) {
        if (c[ci].len < k)
            continue;
        memset(marks[c[ci].genome] + c[ci].start, 1, c[ci].len - k + 1);
        p += c[ci].len - k + 1;
    }
    *npos = p;
}

static uint64_t count_marks(const or_genome *g, uint32_t n, uint8_t **marks)
{
    uint64_t m = 0;
    for (uint32_t gi = 0; gi < n; ++gi)
        for (uint64_t j = 0; j < g[gi].len; ++j)
            m += marks[gi][j] != 0;
    return m;
}

/* Filter-Junctions-Two-Pass (Algorithm 2) on C_in = all positions.
 *   bloom : caller buffer of b/32 words; receives the first-pass filter F
 *   c1    : per genome, n_bases bytes; receives C_temp (marks after pass 1)
 *   c2    : per genome, n_bases bytes; receives C_out (= J(S,k))
 *   with_distinct: also count distinct normalised (k+1)-mers (for the
 *           statistical pins; costs one more sort). */
int or_twopass(const or_genome *g, uint32_t n, uint32_t k, uint64_t b, uint32_t h, uint32_t flags,
               int with_distinct, uint32_t *bloom, uint8_t **c1, uint8_t **c2, or_stats *st)
{
    if (check_args(k, b, h, flags))
        return OR_EINVAL;
    memset(st, 0, sizeof(*st));
    uint64_t nc = 0;
    contig_t *c = make_contigs(g, n, &nc);
    if (!c)
        return OR_ENOMEM;
    vset sent = {0};
    int rc = make_sentinels(g, c, nc, k, flags, &sent);
    if (rc)
        goto out;

    for (uint32_t gi = 0; gi < n; ++gi)
        memset(c1[gi], 0, g[gi].len);
    mark_all(c, nc, k, c1, &st->positions);

    /* first pass: E = Bloom filter of b bits */
    edge_set F = {1, k, h, flags, b, bloom, {0}};
    memset(bloom, 0, (size_t)(b / 32) * sizeof(uint32_t));
    rc = filter_junctions(g, c, nc, k, flags, &sent, &F, c1);
    if (rc)
        goto out;
    st->marks_pass1 = count_marks(g, n, c1);
    for (uint64_t w = 0; w < b / 32; ++w)
        st->bloom_popcount += (uint64_t)__builtin_popcount(bloom[w]);

    /* second pass: E = exact set, starting from the first-pass marks */
    for (uint32_t gi = 0; gi < n; ++gi)
        memcpy(c2[gi], c1[gi], g[gi].len);
    edge_set H = {0, k, h, flags, b, NULL, {0}};
    rc = filter_junctions(g, c, nc, k, flags, &sent, &H, c2);
    st->exact_edges = H.exact.n;
    free(H.exact.v);
    if (rc)
        goto out;
    st->marks_pass2 = count_marks(g, n, c2);

    if (with_distinct) {
        vset all = {0};
        for (uint64_t ci = 0; ci < nc && !rc; ++ci) {
            const uint8_t *s = g[c[ci].genome].codes + c[ci].start;
            for (uint64_t j = 0; j + k + 1 <= c[ci].len; ++j)
                if ((rc = vset_push(&all, norm(s, j, k + 1, flags))))
                    break;
        }
        vset_finish(&all);
        st->distinct_edges = all.n;
        free(all.v);
    }
out:
    free(sent.v);
    free(c);
    return rc;
}

/* ------------------------------------------------------ Algorithm 3 */

/* Multiple Rounds section.  A hash f with range [0, q) splits the normalised
 * k-mers into q subranges; counters e_i estimate |E_i|, the (k+1)-mers that
 * contain a k-mer of subrange i; classes are runs of consecutive subranges
 * formed by a greedy scan; round i runs Algorithm 2 on the positions whose
 * k-mer is in class i.
 *
 * Readings: f(v) = top log2(q) bits of mix64(fold(v) ^ S4), q = 1024.  The
 * counters count (k+1)-mer occurrences, once per distinct subrange among the
 * two k-mers each contains: the text's counting of only first insertions
 * into a Bloom filter depends on insertion order, which a parallel build
 * cannot reproduce, while occurrence counts are order-free.  The scan gives
 * class c the longest run of subranges, at least one while any remain, whose
 * counter sum s satisfies s * l <= sum of all counters; the last class takes
 * every remaining subrange. */
#define OR_Q_LOG2 10u
#define OR_Q (1u << OR_Q_LOG2)
static const uint64_t OR_S4 = 0x452821E638D01377ull; /* hex digits of pi, continued */

static uint32_t subrange_of(kv v, uint32_t k)
{
    return (uint32_t)(or_mix64(fold(v, k) ^ OR_S4) >> (64 - OR_Q_LOG2));
}

static void census(const or_genome *g, const contig_t *c, uint64_t nc, uint32_t k, uint32_t flags,
                   uint64_t *e)
{
    memset(e, 0, OR_Q * sizeof(uint64_t));
    for (uint64_t ci = 0; ci < nc; ++ci) {
        const uint8_t *s = g[c[ci].genome].codes + c[ci].start;
        for (uint64_t j = 0; j + k + 1 <= c[ci].len; ++j) {
            const uint32_t a = subrange_of(norm(s, j, k, flags), k);
            const uint32_t z = subrange_of(norm(s, j + 1, k, flags), k);
            ++e[a];
            if (z != a)
                ++e[z];
        }
    }
}

static void partition(const uint64_t *e, uint32_t l, uint32_t *bound)
{
    unsigned __int128 total = 0;
    for (uint32_t i = 0; i < OR_Q; ++i)
        total += e[i];
    uint32_t next = 0;
    for (uint32_t cls = 0; cls < l; ++cls) {
        bound[cls] = next;
        if (cls == l - 1) {
            next = OR_Q;
            continue;
        }
        unsigned __int128 sum = 0;
        uint32_t taken = 0;
        while (next < OR_Q) {
            const unsigned __int128 with = sum + e[next];
            if (taken > 0 && with * l > total)
                break;
            sum = with;
            ++next;
            ++taken;
        }
    }
    bound[l] = OR_Q;
}

/* Exported for the tests: the partition of given counters. */
void or_partition(const uint64_t *e, uint32_t l, uint32_t *bound)
{
    partition(e, l, bound);
}

/* Exported for the tests: the subrange of a normalised k-mer value (four
 * words, least significant first). */
uint32_t or_subrange(const uint64_t *words, uint32_t k)
{
    return subrange_of(kv_words(words), k);
}

/* Algorithm 3.  bloom receives the last round's filter; c1 the union of the
 * rounds' first-pass marks; c2 the union of their second-pass marks (= J);
 * counters (OR_Q) and bound (l + 1) the census and the partition. */
int or_rounds(const or_genome *g, uint32_t n, uint32_t k, uint64_t b, uint32_t h, uint32_t flags,
              uint32_t l, uint32_t *bloom, uint8_t **c1, uint8_t **c2, or_stats *st,
              uint64_t *counters, uint32_t *bound)
{
    if (check_args(k, b, h, flags) || l < 1 || l > OR_Q)
        return OR_EINVAL;
    memset(st, 0, sizeof(*st));
    uint64_t nc = 0;
    contig_t *c = make_contigs(g, n, &nc);
    if (!c)
        return OR_ENOMEM;
    vset sent = {0};
    uint8_t **ci_marks = calloc(n ? n : 1, sizeof(uint8_t *));
    int rc = ci_marks ? make_sentinels(g, c, nc, k, flags, &sent) : OR_ENOMEM;
    for (uint32_t gi = 0; gi < n && !rc; ++gi)
        if (!(ci_marks[gi] = malloc(g[gi].len ? g[gi].len : 1)))
            rc = OR_ENOMEM;
    if (rc)
        goto out;
    census(g, c, nc, k, flags, counters);
    partition(counters, l, bound);
    for (uint32_t gi = 0; gi < n; ++gi) {
        memset(c1[gi], 0, g[gi].len);
        memset(c2[gi], 0, g[gi].len);
    }
    for (uint32_t r = 0; r < l && !rc; ++r) {
        /* C_r: the positions whose normalised k-mer lies in class r */
        for (uint32_t gi = 0; gi < n; ++gi)
            memset(ci_marks[gi], 0, g[gi].len);
        for (uint64_t x = 0; x < nc; ++x) {
            if (c[x].len < k)
                continue;
            const uint8_t *s = g[c[x].genome].codes + c[x].start;
            uint8_t *C = ci_marks[c[x].genome] + c[x].start;
            for (uint64_t j = 0; j + k <= c[x].len; ++j) {
                const uint32_t sr = subrange_of(norm(s, j, k, flags), k);
                C[j] = sr >= bound[r] && sr < bound[r + 1];
                st->positions += r == 0;
            }
        }
        /* Algorithm 2 from C_r: Bloom pass, then exact pass */
        edge_set F = {1, k, h, flags, b, bloom, {0}};
        memset(bloom, 0, (size_t)(b / 32) * sizeof(uint32_t));
        if ((rc = filter_junctions(g, c, nc, k, flags, &sent, &F, ci_marks)))
            break;
        for (uint64_t w = 0; w < b / 32; ++w)
            st->bloom_popcount += (uint64_t)__builtin_popcount(bloom[w]);
        for (uint32_t gi = 0; gi < n; ++gi)
            for (uint64_t j = 0; j < g[gi].len; ++j)
                c1[gi][j] |= ci_marks[gi][j];
        edge_set H = {0, k, h, flags, b, NULL, {0}};
        rc = filter_junctions(g, c, nc, k, flags, &sent, &H, ci_marks);
        st->exact_edges += H.exact.n;
        free(H.exact.v);
        for (uint32_t gi = 0; gi < n && !rc; ++gi)
            for (uint64_t j = 0; j < g[gi].len; ++j)
                c2[gi][j] |= ci_marks[gi][j];
    }
    if (!rc) {
        st->marks_pass1 = count_marks(g, n, c1);
        st->marks_pass2 = count_marks(g, n, c2);
    }
out:
    if (ci_marks)
        for (uint32_t gi = 0; gi < n; ++gi)
            free(ci_marks[gi]);
    free(ci_marks);
    free(sent.v);
    free(c);
    return rc;
}

/* ------------------------------------------------------ brute force */

/* J(S,k) by the definitions, on G(S) u G(S-bar) (or G(S) alone with the
 * single-strand flag): the edge set is every (k+1)-mer of every string and
 * of every reverse-complement string, taken literally; a vertex is a
 * bifurcation if more than one edge of the set enters or leaves it, a
 * sentinel if it is the first or last k-mer of any of these strings.
 * junction[g][pos] receives 1 at junction positions of the input strings. */
int or_bruteforce(const or_genome *g, uint32_t n, uint32_t k, uint32_t flags, uint8_t **junction)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    uint64_t nc = 0;
    contig_t *c = make_contigs(g, n, &nc);
    if (!c)
        return OR_ENOMEM;
    int rc = OR_OK;
    vset edges = {0}, sent = {0};
    uint8_t buf[130];

    /* the strings of the comprehensive graph */
    uint64_t ns = (flags & OR_SINGLE_STRAND) ? nc : 2 * nc;
    uint8_t **str = (uint8_t **)calloc(ns ? ns : 1, sizeof(uint8_t *));
    uint64_t *slen = (uint64_t *)calloc(ns ? ns : 1, sizeof(uint64_t));
    if (!str || !slen) {
        rc = OR_ENOMEM;
        goto out;
    }
    for (uint64_t ci = 0; ci < nc; ++ci) {
        const uint8_t *s = g[c[ci].genome].codes + c[ci].start;
        uint64_t L = c[ci].len;
        str[ci] = (uint8_t *)malloc(L ? L : 1);
        if (!str[ci]) {
            rc = OR_ENOMEM;
            goto out;
        }
        memcpy(str[ci], s, L);
        slen[ci] = L;
        if (!(flags & OR_SINGLE_STRAND)) {
            uint8_t *r = (uint8_t *)malloc(L ? L : 1);
            if (!r) {
                rc = OR_ENOMEM;
                goto out;
            }
            for (uint64_t t = 0; t < L; ++t)
                r[t] = (uint8_t)(3 - s[L - 1 - t]);
            str[nc + ci] = r;
            slen[nc + ci] = L;
        }
    }
    for (uint64_t si = 0; si < ns; ++si) {
        for (uint64_t j = 0; j + k + 1 <= slen[si]; ++j)
            if ((rc = vset_push(&edges, val(str[si], j, k + 1))))
                goto out;
        if (slen[si] >= k) {
            if ((rc = vset_push(&sent, val(str[si], 0, k))) ||
                (rc = vset_push(&sent, val(str[si], slen[si] - k, k))))
                goto out;
        }
    }
    vset_finish(&edges);
    vset_finish(&sent);

    for (uint32_t gi = 0; gi < n; ++gi)
        memset(junction[gi], 0, g[gi].len);
    for (uint64_t ci = 0; ci < nc; ++ci) {
        const uint8_t *s = str[ci];
        if (slen[ci] < k)
            continue;
        for (uint64_t i = 0; i + k <= slen[ci]; ++i) {
            int in = 0, out = 0;
            for (uint8_t ch = 0; ch < 4; ++ch) {
                memcpy(buf, s + i, k);
                buf[k] = ch;
                out += vset_has(&edges, val(buf, 0, k + 1));
                buf[0] = ch;
                memcpy(buf + 1, s + i, k);
                in += vset_has(&edges, val(buf, 0, k + 1));
            }
            int is_sent = vset_has(&sent, val(s, i, k));
            if (is_sent || in > 1 || out > 1)
                junction[c[ci].genome][c[ci].start + i] = 1;
        }
    }
out:
    if (str)
        for (uint64_t si = 0; si < ns; ++si)
            free(str[si]);
    free(str);
    free(slen);
    free(edges.v);
    free(sent.v);
    free(c);
    return rc;
}

/* --------------------------------------------------- vertices and edges */

/* Vertex id of the k-mer at each given position: its normalised value (four
 * words per position, least significant first) and strand (0 when the k-mer
 * as read is its normalised form). */
void or_vertex(const or_genome *g, uint32_t k, uint32_t flags, const uint64_t *pos, uint64_t npos,
               uint64_t *words, uint8_t *strand)
{
    for (uint64_t i = 0; i < npos; ++i) {
        kv f = val(g->codes, pos[i], k);
        kv r = (flags & OR_SINGLE_STRAND) ? f : rcval(g->codes, pos[i], k);
        const int fwd = kv_cmp(f, r) <= 0;
        const kv m = fwd ? f : r;
        for (int w = 0; w < 4; ++w)
            words[4 * i + w] = m.w[w];
        strand[i] = fwd ? 0 : 1;
    }
}

/* Compacted edges from per-genome junction marks (Reduction section): for
 * every two consecutive junction positions of one string, one edge.
 * Writes up to cap edges as (genome, from, to) triples; returns the count
 * (which may exceed cap: call again with a larger buffer). */
int64_t or_edges(const or_genome *g, uint32_t n, uint32_t k, uint8_t **junction, uint64_t *out,
                 uint64_t cap)
{
    uint64_t nc = 0;
    contig_t *c = make_contigs(g, n, &nc);
    if (!c)
        return OR_ENOMEM;
    uint64_t ne = 0;
    for (uint64_t ci = 0; ci < nc; ++ci) {
        if (c[ci].len < k)
            continue;
        const uint8_t *J = junction[c[ci].genome] + c[ci].start;
        int64_t prev = -1;
        for (uint64_t i = 0; i + k <= c[ci].len; ++i) {
            if (!J[i])
                continue;
            if (prev >= 0) {
                if (ne < cap) {
                    out[3 * ne + 0] = c[ci].genome;
                    out[3 * ne + 1] = c[ci].start + (uint64_t)prev;
                    out[3 * ne + 2] = c[ci].start + i;
                }
                ++ne;
            }
            prev = (int64_t)i;
        }
    }
    free(c);
    return (int64_t)ne;
}

/* ------------------------------------------------- vertices by definition */

/* In- and out-edges of given vertices of the comprehensive graph
 * G(S) u G(S-bar) (G(S) alone with the single-strand flag), straight from the
 * definitions of the Preliminaries section, for inputs too large for
 * or_bruteforce: every (k+1)-mer of every string is an edge, and so is its
 * reverse complement; an edge leaves the vertex spelled by its first k bases
 * and enters the one spelled by its last k bases.  A vertex is a sentinel
 * when it is the first or last k-mer of a string of S or of S-bar.
 *
 * The query vertices are literal k-mer values (not normalised).  For vertex
 * v, bit c of in_mask[v] is set when c.v is an edge, bit c of out_mask[v]
 * when v.c is one, and sent[v] when v is a sentinel.
 *
 * One streaming pass: along each string the k-mer at position i and its
 * reverse complement are rolled by one base per step and looked up in a hash
 * set of the query vertices.  The edge s[i-1..i+k-1] enters the k-mer v at i
 * by base s[i-1], and its reverse complement leaves rc(v) by base comp(s[i-1]);
 * the edge s[i..i+k] leaves v by base s[i+k], and its reverse complement
 * enters rc(v) by base comp(s[i+k]).  Strings are cut into pieces that worker
 * threads take in turn, each with its own masks, ORed together at the end
 * (the masks are sets, so the order does not matter). */

typedef struct {
    kv *key;
    int64_t *idx; /* query index, -1 = empty slot */
    uint64_t mask;
    uint64_t *pre; /* one bit per hash value prefix: a quick "not in the set" */
    uint32_t pre_log2;
    uint32_t k;
} vtable;

static const uint64_t OR_S5 = 0xBE5466CF34E90C6Cull; /* hex digits of pi, continued */

static uint64_t vhash(kv v, uint32_t k)
{
    return or_mix64(fold(v, k) ^ OR_S5);
}

static int vtable_init(vtable *t, const kv *vals, uint64_t nv, uint32_t k)
{
    uint64_t cap = 1024;
    while (cap < 2 * nv)
        cap *= 2;
    t->k = k;
    t->mask = cap - 1;
    t->pre_log2 = 10;
    while ((1ull << t->pre_log2) < 16 * nv && t->pre_log2 < 30)
        ++t->pre_log2;
    t->key = (kv *)malloc(cap * sizeof(kv));
    t->idx = (int64_t *)malloc(cap * sizeof(int64_t));
    t->pre = (uint64_t *)calloc((1ull << t->pre_log2) / 64 + 1, sizeof(uint64_t));
    if (!t->key || !t->idx || !t->pre)
        return OR_ENOMEM;
    for (uint64_t i = 0; i < cap; ++i)
        t->idx[i] = -1;
    for (uint64_t q = 0; q < nv; ++q) {
        const uint64_t h = vhash(vals[q], k);
        const uint64_t b = h >> (64 - t->pre_log2);
        t->pre[b >> 6] |= 1ull << (b & 63);
        uint64_t s = h & t->mask;
        while (t->idx[s] >= 0 && kv_cmp(t->key[s], vals[q]) != 0)
            s = (s + 1) & t->mask;
        if (t->idx[s] < 0) {
            t->key[s] = vals[q];
            t->idx[s] = (int64_t)q;
        }
    }
    return OR_OK;
}

static void vtable_free(vtable *t)
{
    free(t->key);
    free(t->idx);
    free(t->pre);
}

/* Index of the query vertex with value v (its first listing), or -1. */
static int64_t vtable_find(const vtable *t, kv v)
{
    const uint64_t h = vhash(v, t->k);
    const uint64_t b = h >> (64 - t->pre_log2);
    if (!((t->pre[b >> 6] >> (b & 63)) & 1))
        return -1;
    for (uint64_t s = h & t->mask; t->idx[s] >= 0; s = (s + 1) & t->mask)
        if (kv_cmp(t->key[s], v) == 0)
            return t->idx[s];
    return -1;
}

/* v = v / 4 (drop the last base), then put base c in front of L-1 bases. */
static void kv_push_front(kv *v, uint8_t c, uint32_t L)
{
    v->w[0] = (v->w[0] >> 2) | (v->w[1] << 62);
    v->w[1] = (v->w[1] >> 2) | (v->w[2] << 62);
    v->w[2] = (v->w[2] >> 2) | (v->w[3] << 62);
    v->w[3] >>= 2;
    const uint32_t bit = 2 * (L - 1);
    v->w[bit >> 6] |= (uint64_t)c << (bit & 63);
}

/* Keep the low 2L bits of v. */
static void kv_trim(kv *v, uint32_t L)
{
    for (uint32_t i = 0; i < 4; ++i) {
        const uint32_t lo = 64 * i;
        if (2 * L <= lo)
            v->w[i] = 0;
        else if (2 * L < lo + 64)
            v->w[i] &= (1ull << (2 * L - lo)) - 1;
    }
}

/* A genome as packed 2-bit bases plus N runs (the library's input format):
 * base j in byte j >> 2 at bits 2 (j & 3). */
typedef struct {
    const uint8_t *packed;
    uint64_t n_bases;
    const uint64_t *n_runs; /* (start, length) pairs, sorted */
    uint64_t n_nruns;
} or_packed_genome;

/* A piece of work: positions [p0, p1) of one string.  The string's bases
 * are codes[start ...] (codes input) or packed[start ...] (packed input). */
typedef struct {
    const uint8_t *codes;  /* NULL for packed input */
    const uint8_t *packed;
    uint64_t start, len;   /* string in genome coordinates */
    uint64_t p0, p1;
} vm_piece;

typedef struct {
    const vm_piece *pieces;
    uint64_t n_pieces;
    uint64_t next; /* shared cursor */
    const vtable *t;
    uint32_t k, single;
    uint64_t nv;
    int rc;
} vm_job;

typedef struct {
    vm_job *job;
    uint8_t *in, *out, *sent;
} vm_worker;

#define VM_PIECE 4000000ull

static uint8_t base_of(const vm_piece *pc, uint64_t j) /* j relative to the string */
{
    const uint64_t a = pc->start + j;
    if (pc->codes)
        return pc->codes[a];
    return (uint8_t)((pc->packed[a >> 2] >> (2 * (a & 3))) & 3);
}

static void *vm_run(void *arg)
{
    vm_worker *wk = (vm_worker *)arg;
    vm_job *J = wk->job;
    const uint32_t k = J->k;
    uint8_t *buf = (uint8_t *)malloc(VM_PIECE + 2 * k + 2);
    if (!buf) {
        __atomic_store_n(&J->rc, OR_ENOMEM, __ATOMIC_RELAXED);
        return NULL;
    }
    for (;;) {
        const uint64_t pi = __atomic_fetch_add(&J->next, 1, __ATOMIC_RELAXED);
        if (pi >= J->n_pieces)
            break;
        const vm_piece *pc = &J->pieces[pi];
        /* bases from p0 - 1 (predecessor) to p1 + k (successor of the last
         * position), clipped to the string; buf[i - lo] is base i */
        const uint64_t lo = pc->p0 ? pc->p0 - 1 : 0;
        const uint64_t hi = pc->p1 + k < pc->len ? pc->p1 + k + 1 : pc->len;
        for (uint64_t j = lo; j < hi; ++j)
            buf[j - lo] = base_of(pc, j);
#define B(i) buf[(i) - lo] /* base i of the string */
        kv f = val(buf, pc->p0 - lo, k), r = rcval(buf, pc->p0 - lo, k);
        const uint64_t last = pc->len - k;
        for (uint64_t i = pc->p0; i < pc->p1; ++i) {
            const int64_t qf = vtable_find(J->t, f);
            const int64_t qr = J->single ? -1 : vtable_find(J->t, r);
            if (qf >= 0 || qr >= 0) {
                const int end = i == 0 || i == last;
                if (qf >= 0) {
                    if (end)
                        wk->sent[qf] = 1;
                    if (i > 0)
                        wk->in[qf] |= (uint8_t)(1u << B(i - 1));
                    if (i < last)
                        wk->out[qf] |= (uint8_t)(1u << B(i + k));
                }
                if (qr >= 0) {
                    if (end)
                        wk->sent[qr] = 1;
                    if (i > 0)
                        wk->out[qr] |= (uint8_t)(1u << (3 - B(i - 1)));
                    if (i < last)
                        wk->in[qr] |= (uint8_t)(1u << (3 - B(i + k)));
                }
            }
            if (i < last) {
                kv_push(&f, B(i + k));
                kv_trim(&f, k);
                kv_push_front(&r, (uint8_t)(3 - B(i + k)), k);
            }
        }
    }
#undef B
    free(buf);
    return NULL;
}

/* Pieces of every string of length >= k; strings come from make_contigs
 * (codes) or from the N runs (packed). */
static int add_pieces(vm_piece **pcs, uint64_t *n, uint64_t *cap, const uint8_t *codes,
                      const uint8_t *packed, uint64_t start, uint64_t len, uint32_t k)
{
    if (len < k)
        return OR_OK;
    const uint64_t npos = len - k + 1;
    for (uint64_t p0 = 0; p0 < npos; p0 += VM_PIECE) {
        if (*n == *cap) {
            uint64_t nc = *cap ? 2 * *cap : 256;
            vm_piece *np = (vm_piece *)realloc(*pcs, nc * sizeof(vm_piece));
            if (!np)
                return OR_ENOMEM;
            *pcs = np;
            *cap = nc;
        }
        vm_piece *pc = &(*pcs)[(*n)++];
        pc->codes = codes;
        pc->packed = packed;
        pc->start = start;
        pc->len = len;
        pc->p0 = p0;
        pc->p1 = p0 + VM_PIECE < npos ? p0 + VM_PIECE : npos;
    }
    return OR_OK;
}

static int run_vertex_masks(vm_piece *pcs, uint64_t npc, uint32_t k, uint32_t flags,
                            const uint64_t *vwords, uint64_t nv, uint8_t *in_mask,
                            uint8_t *out_mask, uint8_t *sent, uint32_t threads)
{
    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    kv *vals = (kv *)malloc((nv ? nv : 1) * sizeof(kv));
    if (!vals)
        return OR_ENOMEM;
    for (uint64_t q = 0; q < nv; ++q)
        vals[q] = kv_words(vwords + 4 * q);
    vtable t;
    memset(&t, 0, sizeof(t));
    int rc = vtable_init(&t, vals, nv, k);
    vm_job job = {pcs, npc, 0, &t, k, (flags & OR_SINGLE_STRAND) ? 1u : 0u, nv, OR_OK};
    vm_worker *wk = (vm_worker *)calloc(threads, sizeof(vm_worker));
    pthread_t *th = (pthread_t *)calloc(threads, sizeof(pthread_t));
    if (!rc && (!wk || !th))
        rc = OR_ENOMEM;
    uint32_t started = 0;
    for (uint32_t i = 0; i < threads && !rc; ++i) {
        wk[i].job = &job;
        wk[i].in = (uint8_t *)calloc(nv ? nv : 1, 1);
        wk[i].out = (uint8_t *)calloc(nv ? nv : 1, 1);
        wk[i].sent = (uint8_t *)calloc(nv ? nv : 1, 1);
        if (!wk[i].in || !wk[i].out || !wk[i].sent)
            rc = OR_ENOMEM;
    }
    for (uint32_t i = 0; i < threads && !rc; ++i, ++started)
        if (pthread_create(&th[i], NULL, vm_run, &wk[i]))
            break;
    if (!rc && started == 0)
        rc = OR_ENOMEM;
    for (uint32_t i = 0; i < started; ++i)
        pthread_join(th[i], NULL);
    if (!rc)
        rc = job.rc;
    if (!rc) {
        /* a value listed twice shares its first listing's masks */
        memset(in_mask, 0, nv);
        memset(out_mask, 0, nv);
        memset(sent, 0, nv);
        for (uint32_t i = 0; i < started; ++i)
            for (uint64_t q = 0; q < nv; ++q) {
                in_mask[q] |= wk[i].in[q];
                out_mask[q] |= wk[i].out[q];
                sent[q] |= wk[i].sent[q];
            }
        for (uint64_t q = 0; q < nv; ++q) {
            const int64_t f = vtable_find(&t, vals[q]);
            in_mask[q] = in_mask[f];
            out_mask[q] = out_mask[f];
            sent[q] = sent[f];
        }
    }
    if (wk)
        for (uint32_t i = 0; i < threads; ++i) {
            free(wk[i].in);
            free(wk[i].out);
            free(wk[i].sent);
        }
    free(wk);
    free(th);
    vtable_free(&t);
    free(vals);
    return rc;
}

/* vwords: 4 words per query vertex (literal value, least significant word
 * first); in_mask, out_mask, sent: nv bytes each. */
int or_vertex_masks(const or_genome *g, uint32_t n, uint32_t k, uint32_t flags,
                    const uint64_t *vwords, uint64_t nv, uint8_t *in_mask, uint8_t *out_mask,
                    uint8_t *sent, uint32_t threads)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    uint64_t nc = 0;
    contig_t *c = make_contigs(g, n, &nc);
    if (!c)
        return OR_ENOMEM;
    vm_piece *pcs = NULL;
    uint64_t npc = 0, cap = 0;
    int rc = OR_OK;
    for (uint64_t ci = 0; ci < nc && !rc; ++ci)
        rc = add_pieces(&pcs, &npc, &cap, g[c[ci].genome].codes, NULL, c[ci].start, c[ci].len, k);
    if (!rc)
        rc = run_vertex_masks(pcs, npc, k, flags, vwords, nv, in_mask, out_mask, sent, threads);
    free(pcs);
    free(c);
    return rc;
}

/* The same on packed genomes (strings = the complement of the N runs). */
int or_vertex_masks_packed(const or_packed_genome *g, uint32_t n, uint32_t k, uint32_t flags,
                           const uint64_t *vwords, uint64_t nv, uint8_t *in_mask,
                           uint8_t *out_mask, uint8_t *sent, uint32_t threads)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    vm_piece *pcs = NULL;
    uint64_t npc = 0, cap = 0;
    int rc = OR_OK;
    for (uint32_t gi = 0; gi < n && !rc; ++gi) {
        uint64_t from = 0;
        for (uint64_t r = 0; r <= g[gi].n_nruns && !rc; ++r) {
            const uint64_t to = r < g[gi].n_nruns ? g[gi].n_runs[2 * r] : g[gi].n_bases;
            if (to < from || to > g[gi].n_bases)
                rc = OR_EINVAL;
            else
                rc = add_pieces(&pcs, &npc, &cap, NULL, g[gi].packed, from, to - from, k);
            if (r < g[gi].n_nruns)
                from = to + g[gi].n_runs[2 * r + 1];
        }
    }
    if (!rc)
        rc = run_vertex_masks(pcs, npc, k, flags, vwords, nv, in_mask, out_mask, sent, threads);
    free(pcs);
    return rc;
}

/* Junction status of sampled positions (samp_g[i], samp_pos[i], each a k-mer
 * start inside a string): a junction is a sentinel or a vertex with more than
 * one in- or out-edge (Preliminaries section), the edges taken from
 * or_vertex_masks.  status[i] receives 1 for a junction. */
static int status_from_masks(uint64_t ns, const uint64_t *vw, uint32_t k, uint32_t flags,
                             int (*masks)(const void *, uint32_t, uint32_t, uint32_t,
                                          const uint64_t *, uint64_t, uint8_t *, uint8_t *,
                                          uint8_t *, uint32_t),
                             const void *g, uint32_t n, uint8_t *status, uint32_t threads)
{
    uint8_t *in = (uint8_t *)malloc(ns ? ns : 1), *out = (uint8_t *)malloc(ns ? ns : 1),
            *sent = (uint8_t *)malloc(ns ? ns : 1);
    int rc = (in && out && sent) ? OR_OK : OR_ENOMEM;
    if (!rc)
        rc = masks(g, n, k, flags, vw, ns, in, out, sent, threads);
    for (uint64_t i = 0; i < ns && !rc; ++i)
        status[i] = (uint8_t)(sent[i] || __builtin_popcount(in[i]) > 1 ||
                              __builtin_popcount(out[i]) > 1);
    free(in);
    free(out);
    free(sent);
    return rc;
}

static int masks_codes(const void *g, uint32_t n, uint32_t k, uint32_t flags, const uint64_t *vw,
                       uint64_t nv, uint8_t *in, uint8_t *out, uint8_t *sent, uint32_t threads)
{
    return or_vertex_masks((const or_genome *)g, n, k, flags, vw, nv, in, out, sent, threads);
}

static int masks_packed(const void *g, uint32_t n, uint32_t k, uint32_t flags, const uint64_t *vw,
                        uint64_t nv, uint8_t *in, uint8_t *out, uint8_t *sent, uint32_t threads)
{
    return or_vertex_masks_packed((const or_packed_genome *)g, n, k, flags, vw, nv, in, out, sent,
                                  threads);
}

int or_sample_status(const or_genome *g, uint32_t n, uint32_t k, uint32_t flags,
                     const uint32_t *samp_g, const uint64_t *samp_pos, uint64_t ns, uint8_t *status,
                     uint32_t threads)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    uint64_t *vw = (uint64_t *)malloc((ns ? ns : 1) * 4 * sizeof(uint64_t));
    if (!vw)
        return OR_ENOMEM;
    for (uint64_t i = 0; i < ns; ++i) {
        const kv v = val(g[samp_g[i]].codes, samp_pos[i], k);
        memcpy(vw + 4 * i, v.w, sizeof(v.w));
    }
    int rc = status_from_masks(ns, vw, k, flags, masks_codes, g, n, status, threads);
    free(vw);
    return rc;
}

int or_sample_status_packed(const or_packed_genome *g, uint32_t n, uint32_t k, uint32_t flags,
                            const uint32_t *samp_g, const uint64_t *samp_pos, uint64_t ns,
                            uint8_t *status, uint32_t threads)
{
    if (k < 1 || k > 127)
        return OR_EINVAL;
    uint64_t *vw = (uint64_t *)malloc((ns ? ns : 1) * 4 * sizeof(uint64_t));
    if (!vw)
        return OR_ENOMEM;
    for (uint64_t i = 0; i < ns; ++i) {
        kv v = kv_zero();
        for (uint32_t t = 0; t < k; ++t) {
            const uint64_t a = samp_pos[i] + t;
            kv_push(&v, (uint8_t)((g[samp_g[i]].packed[a >> 2] >> (2 * (a & 3))) & 3));
        }
        memcpy(vw + 4 * i, v.w, sizeof(v.w));
    }
    int rc = status_from_masks(ns, vw, k, flags, masks_packed, g, n, status, threads);
    free(vw);
    return rc;
}
