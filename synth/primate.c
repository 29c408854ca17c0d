/* Seeded generator of the primate-scale workload (8 genomes of 3 Gbp from one
 * random base).  An input tool shared by the oracle tests and the GPU tests
 * and benchmarks; it holds none of the junction-finding arithmetic.  Written
 * in C because generating 24 Gbp with numpy takes minutes.
 *
 * Recipe (all lengths and counts multiplied by `scale`, counts at least 1):
 *   base      L = 3e9 uniform i.i.d. bases, drawn per 2^20-base region from
 *             its own stream (so the result is independent of thread count);
 *   repeats   written over the base at uniform offsets, in order: 1e6 copies
 *             of one 300 bp family consensus, then 1e5 copies of one 6 kbp
 *             consensus, each copy at its own divergence d ~ U[10%, 20%]
 *             (every base independently substituted with probability d by
 *             one of the other three, uniformly);
 *   genome g  (g = 0..7) the base with SNPs at rate d_g = 0.5% + g * 3.5% / 7
 *             (same substitution rule; genomes g and g' differ by about
 *             d_g + d_g': 1% to 8%), then indel events at rate d_g / 10 per
 *             base (half insertions of uniform bases before the base at the
 *             event, half deletions starting there; length U{1..10}; events
 *             falling inside a deletion are dropped), then 300 runs of N of
 *             length U{1000..10000} at uniform offsets.
 *
 * Randomness: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014); the stream of
 * (seed, genome, region) starts from the SplitMix64 output of
 * seed ^ genome << 32 ^ region.  Event positions use geometric gaps.
 * Codes: A=0 C=1 G=2 T=3 N=4.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BASE_STREAM 0xFFFFu
#define REPEAT_STREAM 0xFFFEu
#define REGION_LOG2 20

typedef struct {
    uint64_t s;
} rng_t;

static uint64_t sm64(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static rng_t stream(uint64_t seed, uint64_t genome, uint64_t region)
{
    uint64_t s = seed ^ (genome << 32) ^ region;
    rng_t r = {sm64(&s)};
    return r;
}

static uint64_t next(rng_t *r) { return sm64(&r->s); }

/* uniform in [0, 1) with 53 bits */
static double unif(rng_t *r) { return (double)(next(r) >> 11) * (1.0 / 9007199254740992.0); }

/* uniform integer in [lo, hi] */
static uint64_t unif_int(rng_t *r, uint64_t lo, uint64_t hi)
{
    return lo + next(r) % (hi - lo + 1);
}

/* gap to the next event of a Bernoulli(p) process: P(gap = i) = (1-p)^i p */
static uint64_t geo_gap(rng_t *r, double p)
{
    if (p <= 0)
        return UINT64_MAX / 2;
    if (p >= 1)
        return 0;
    double u = unif(r);
    if (u <= 0)
        u = 1e-300;
    return (uint64_t)floor(log(u) / log1p(-p));
}

static uint8_t other_base(rng_t *r, uint8_t b) { return (uint8_t)((b + 1 + next(r) % 3) & 3); }

static uint64_t scaled(double n, double scale)
{
    double v = floor(n * scale + 0.5);
    return v < 1 ? 1 : (uint64_t)v;
}

uint64_t syn_primate_base_len(double scale) { return scaled(3e9, scale); }

/* the base genome, repeats included, into base[syn_primate_base_len(scale)] */
void syn_primate_base(uint64_t seed, double scale, uint8_t *base)
{
    const uint64_t L = syn_primate_base_len(scale);
    for (uint64_t r0 = 0; r0 < L; r0 += 1ull << REGION_LOG2) {
        rng_t r = stream(seed, BASE_STREAM, r0 >> REGION_LOG2);
        const uint64_t end = r0 + (1ull << REGION_LOG2) < L ? r0 + (1ull << REGION_LOG2) : L;
        for (uint64_t i = r0; i < end; i += 32) {
            uint64_t x = next(&r);
            for (uint64_t j = i; j < end && j < i + 32; ++j, x >>= 2)
                base[j] = (uint8_t)(x & 3);
        }
    }
    const struct {
        uint64_t len;
        double copies;
    } fam[2] = {{300, 1e6}, {6000, 1e5}};
    uint8_t *cons = (uint8_t *)malloc(6000);
    if (!cons)
        abort();
    for (int f = 0; f < 2; ++f) {
        const uint64_t len = fam[f].len < L ? fam[f].len : L;
        rng_t rc = stream(seed, REPEAT_STREAM, (uint64_t)f << 40);
        for (uint64_t j = 0; j < len; ++j)
            cons[j] = (uint8_t)(next(&rc) & 3);
        const uint64_t n = scaled(fam[f].copies, scale);
        for (uint64_t c = 0; c < n; ++c) {
            rng_t r = stream(seed, REPEAT_STREAM, ((uint64_t)f << 40) | (c + 1));
            const uint64_t at = unif_int(&r, 0, L - len);
            const double d = 0.10 + 0.10 * unif(&r);
            memcpy(base + at, cons, len);
            for (uint64_t j = geo_gap(&r, d); j < len; j += 1 + geo_gap(&r, d))
                base[at + j] = other_base(&r, base[at + j]);
        }
    }
    free(cons);
}

/* Room genome g needs: its output length never exceeds this. */
uint64_t syn_primate_genome_cap(uint64_t L, uint32_t g)
{
    const double d = 0.005 + g * 0.035 / 7;
    /* insertions add at most 10 bases per event; events at rate d/10 */
    return L + (uint64_t)(L * d * 1.2) + 4096;
}

/* Genome g from the base; returns its length (written to out[0..cap)), or 0
 * when cap is too small. */
uint64_t syn_primate_genome(const uint8_t *base, uint64_t L, uint64_t seed, double scale,
                            uint32_t g, uint8_t *out, uint64_t cap)
{
    const double d = 0.005 + g * 0.035 / 7, di = d / 10;
    rng_t rs = stream(seed, g, 1), ri = stream(seed, g, 2), rn = stream(seed, g, 3);
    uint64_t snp = geo_gap(&rs, d), ev = geo_gap(&ri, di), n = 0, p = 0;
    while (p < L) {
        /* copy up to the next event */
        uint64_t stop = snp < ev ? snp : ev;
        if (stop > L)
            stop = L;
        if (stop > p) {
            if (n + (stop - p) > cap)
                return 0;
            memcpy(out + n, base + p, stop - p);
            n += stop - p;
            p = stop;
            continue;
        }
        if (ev == p) {
            const int ins = (int)(next(&ri) & 1);
            const uint64_t len = unif_int(&ri, 1, 10);
            if (ins) {
                if (n + len > cap)
                    return 0;
                for (uint64_t j = 0; j < len; ++j)
                    out[n++] = (uint8_t)(next(&ri) & 3);
                ev = p + 1 + geo_gap(&ri, di);
            } else {
                p += len;
                /* events inside the deletion are dropped */
                ev = p + geo_gap(&ri, di);
                while (snp < p)
                    snp += 1 + geo_gap(&rs, d);
            }
            continue;
        }
        /* snp == p */
        if (n + 1 > cap)
            return 0;
        out[n++] = other_base(&rs, base[p]);
        ++p;
        snp = p + geo_gap(&rs, d);
    }
    const uint64_t runs = scaled(300, scale);
    for (uint64_t i = 0; i < runs; ++i) {
        const uint64_t len = unif_int(&rn, 1000, 10000);
        if (len >= n)
            break;
        const uint64_t at = unif_int(&rn, 0, n - len);
        memset(out + at, 4, len);
    }
    return n;
}

/* 2-bit packing (base j in byte j >> 2 at bits 2 (j & 3), N stored as 0) and
 * the N runs as (start, length) pairs; returns the number of runs, or
 * UINT64_MAX when more than max_runs. */
uint64_t syn_pack(const uint8_t *codes, uint64_t n, uint8_t *packed, uint64_t *runs,
                  uint64_t max_runs)
{
    memset(packed, 0, (n + 3) / 4);
    uint64_t nr = 0, start = 0;
    int in_n = 0;
    for (uint64_t j = 0; j < n; ++j) {
        const uint8_t c = codes[j];
        if (c > 3) {
            if (!in_n) {
                in_n = 1;
                start = j;
            }
            continue;
        }
        if (in_n) {
            if (nr == max_runs)
                return UINT64_MAX;
            runs[2 * nr] = start;
            runs[2 * nr + 1] = j - start;
            ++nr;
            in_n = 0;
        }
        packed[j >> 2] |= (uint8_t)(c << (2 * (j & 3)));
    }
    if (in_n) {
        if (nr == max_runs)
            return UINT64_MAX;
        runs[2 * nr] = start;
        runs[2 * nr + 1] = n - start;
        ++nr;
    }
    return nr;
}
