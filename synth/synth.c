/*
 * synth.c -- seeded, counter-based synthetic genomes and query sets.
 *
 * Input generation only: this file draws random contig lengths, GC content,
 * bases, N positions and query sequences. It holds none of the alignment
 * method's arithmetic (no window comparison, no mismatch counting, no
 * reverse complement of queries), and both the product path and the oracle
 * consume its output as plain ASCII bytes. For a producer that hands the
 * scan packed input, the same bases are also written as the two 2-bit code
 * planes of that input format (synth_fill_packed).
 *
 * Randomness: SplitMix64 (Steele, Lea & Flood 2014), used two ways:
 *   - key(seed, stream, a, b) mixes four integers into a 64-bit state with the
 *     SplitMix64 finaliser, so any (contig, block) can be regenerated without
 *     generating what comes before it;
 *   - from that state the ordinary SplitMix64 sequence (state += golden gamma,
 *     output = finaliser(state)) supplies the draws inside a block.
 *
 * Streams: 1 contig lengths, 2 contig GC, 3 bases, 4 iid N, 5 N runs,
 *          6 queries.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#if defined(__x86_64__)
#include <immintrin.h>
#endif

#define SYN_GAMMA 0x9E3779B97F4A7C15ULL
#define SYN_BLOCK 4096ULL

static inline uint64_t syn_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t syn_key(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b)
{
    uint64_t z = syn_fin(seed * SYN_GAMMA + stream + 1);
    z = syn_fin(z + (a + 1) * SYN_GAMMA);
    z = syn_fin(z + (b + 1) * SYN_GAMMA);
    return z;
}

typedef struct { uint64_t s; } syn_rng;

static inline uint64_t syn_next(syn_rng *r)
{
    r->s += SYN_GAMMA;
    return syn_fin(r->s);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double syn_unif(syn_rng *r)
{
    return (double)(syn_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

/* raw SplitMix64 sequence from a seed; exported so tests can check the
 * generator against the published reference outputs */
void synth_splitmix64(uint64_t seed, uint64_t n, uint64_t *out)
{
    syn_rng r = { seed };
    for (uint64_t i = 0; i < n; i++) out[i] = syn_next(&r);
}

/* ------------------------------------------------------------------ */
/* contig table                                                        */
/* ------------------------------------------------------------------ */

/*
 * Contig lengths.
 *   mode 0: fixed -- n_fixed contigs of fixed_len each (total ignored)
 *   mode 1: lognormal(median, sigma), lengths below min_len raised to min_len,
 *           contigs added until `total` bases; the last one truncated so the
 *           lengths sum to exactly `total`
 *   mode 2: lognormal(median, sigma) redrawn until inside [min_len, max_len],
 *           same total rule as mode 1
 * Writes at most `cap` lengths; returns the number of contigs, or -1 when
 * `cap` is too small.
 */
int64_t synth_contig_lengths(uint64_t seed, int mode, uint64_t n_fixed, uint64_t fixed_len,
                             double median, double sigma, uint64_t min_len, uint64_t max_len,
                             uint64_t total, uint64_t *out, int64_t cap)
{
    if (mode == 0) {
        if ((int64_t)n_fixed > cap) return -1;
        for (uint64_t i = 0; i < n_fixed; i++) out[i] = fixed_len;
        return (int64_t)n_fixed;
    }
    uint64_t sum = 0;
    int64_t n = 0;
    while (sum < total) {
        if (n >= cap) return -1;
        syn_rng r = { syn_key(seed, 1, (uint64_t)n, 0) };
        double len;
        for (;;) {
            /* Box-Muller standard normal */
            double u1 = syn_unif(&r), u2 = syn_unif(&r);
            if (u1 < 1e-300) u1 = 1e-300;
            double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
            len = median * exp(sigma * z);
            if (mode == 1) {
                if (len < (double)min_len) len = (double)min_len;
                break;
            }
            if (len >= (double)min_len && len <= (double)max_len) break;
        }
        uint64_t L = (uint64_t)llround(len);
        if (L < 1) L = 1;
        if (sum + L > total) L = total - sum;
        out[n++] = L;
        sum += L;
    }
    return n;
}

/* per-contig GC fraction, uniform in [gc_lo, gc_hi) */
void synth_contig_gc(uint64_t seed, uint64_t first, uint64_t n, double gc_lo, double gc_hi,
                     double *out)
{
    for (uint64_t i = 0; i < n; i++) {
        syn_rng r = { syn_key(seed, 2, first + i, 0) };
        out[i] = gc_lo + (gc_hi - gc_lo) * syn_unif(&r);
    }
}

/* ------------------------------------------------------------------ */
/* bases                                                               */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t seed;
    int n_mode;          /* 0 no N, 1 each base N with prob n_param, 2 N runs */
    double n_param;      /* mode 1: per-base probability; mode 2: N fraction */
    uint32_t run_min;    /* mode 2: run length uniform in [run_min, run_max] */
    uint32_t run_max;
} syn_spec;

/* fill out[0..n) with bases [x0, x0+n) of contig `c` (length clen, GC gc) */
/* AVX2 path for whole draws (4 draws = 32 bases per step), the same draws and
 * the same byte mapping as the scalar loop; synth_set_simd(0) turns it off
 * (the tests compare both). */
static int syn_simd = 1;

void synth_set_simd(int on) { syn_simd = on; }

#if defined(__x86_64__)
__attribute__((target("avx2"))) static inline __m256i syn_mul64(__m256i z, uint64_t c)
{
    const __m256i clo = _mm256_set1_epi64x((long long)(c & 0xFFFFFFFFULL));
    const __m256i chi = _mm256_set1_epi64x((long long)(c >> 32));
    const __m256i lo = _mm256_mul_epu32(z, clo);
    const __m256i t1 = _mm256_mul_epu32(_mm256_srli_epi64(z, 32), clo);
    const __m256i t2 = _mm256_mul_epu32(z, chi);
    return _mm256_add_epi64(lo, _mm256_slli_epi64(_mm256_add_epi64(t1, t2), 32));
}

/* whole draws from state *s (advanced), 8 bases each, into o; returns draws done */
__attribute__((target("avx2"))) static uint64_t fill_draws_avx2(uint64_t *s, uint64_t draws,
                                                               uint32_t thr, uint8_t *o)
{
    const __m256i g = _mm256_set_epi64x((long long)(4 * SYN_GAMMA), (long long)(3 * SYN_GAMMA),
                                        (long long)(2 * SYN_GAMMA), (long long)SYN_GAMMA);
    const __m256i step = _mm256_set1_epi64x((long long)(4 * SYN_GAMMA));
    const __m256i m7 = _mm256_set1_epi8(0x7F), vthr = _mm256_set1_epi8((char)thr);
    const __m256i cc = _mm256_set1_epi8('C'), cg = _mm256_set1_epi8('G');
    const __m256i ca = _mm256_set1_epi8('A'), ct = _mm256_set1_epi8('T');
    __m256i st = _mm256_add_epi64(_mm256_set1_epi64x((long long)*s), g);
    uint64_t done = 0;
    for (; done + 4 <= draws; done += 4) {
        __m256i z = st;
        z = syn_mul64(_mm256_xor_si256(z, _mm256_srli_epi64(z, 30)), 0xBF58476D1CE4E5B9ULL);
        z = syn_mul64(_mm256_xor_si256(z, _mm256_srli_epi64(z, 27)), 0x94D049BB133111EBULL);
        z = _mm256_xor_si256(z, _mm256_srli_epi64(z, 31));
        const __m256i low7 = _mm256_and_si256(z, m7);
        /* A/T where low7 >= thr (unsigned), G/C otherwise; the top bit picks G or T */
        const __m256i at = _mm256_cmpeq_epi8(_mm256_max_epu8(low7, vthr), low7);
        const __m256i gcb = _mm256_blendv_epi8(cc, cg, z);
        const __m256i atb = _mm256_blendv_epi8(ca, ct, z);
        _mm256_storeu_si256((__m256i *)(o + 8 * done), _mm256_blendv_epi8(gcb, atb, at));
        st = _mm256_add_epi64(st, step);
    }
    *s += done * SYN_GAMMA;
    return done;
}
#endif

static void fill_range(const syn_spec *sp, uint64_t c, uint64_t clen, double gc,
                       uint64_t x0, uint64_t n, uint8_t *out)
{
    if (x0 >= clen) return;
    if (x0 + n > clen) n = clen - x0;
    /* 8 random bits per base: the low 7 against the GC fraction (so GC is
     * quantised to 1/128), the top bit picks G/C or A/T */
    const uint32_t thr = (uint32_t)(gc * 128.0 + 0.5);
    uint8_t table[256];
    for (uint32_t u = 0; u < 256; u++)
        table[u] = (u & 0x7Fu) < thr ? ((u >> 7) ? 'G' : 'C') : ((u >> 7) ? 'T' : 'A');
    uint64_t x = x0, end = x0 + n;
    while (x < end) {
        uint64_t blk = x / SYN_BLOCK;
        uint64_t bstart = blk * SYN_BLOCK;
        uint64_t bend = bstart + SYN_BLOCK;
        if (bend > end) bend = end;
        syn_rng r = { syn_key(sp->seed, 3, c, blk) };
        /* skip draws for the part of the block before x: 8 bases per draw */
        uint64_t skip = (x - bstart) / 8;
        r.s += skip * SYN_GAMMA;
        uint64_t pos = bstart + skip * 8;
        if (pos < x || bend - pos < 8) {
            /* ragged head or tail: base by base */
            while (pos < bend) {
                uint64_t v = syn_next(&r);
                for (int j = 0; j < 8 && pos < bend; j++, pos++)
                    if (pos >= x) out[pos - x0] = table[(v >> (8 * j)) & 0xFFu];
            }
        }
        /* whole draws */
        uint8_t *o = out + (pos - x0);
#if defined(__x86_64__)
        if (syn_simd && __builtin_cpu_supports("avx2")) {
            const uint64_t done = fill_draws_avx2(&r.s, (bend - pos) / 8, thr, o);
            o += 8 * done;
            pos += 8 * done;
        }
#endif
        while (pos + 8 <= bend) {
            uint64_t v = syn_next(&r);
            o[0] = table[v & 0xFF];
            o[1] = table[(v >> 8) & 0xFF];
            o[2] = table[(v >> 16) & 0xFF];
            o[3] = table[(v >> 24) & 0xFF];
            o[4] = table[(v >> 32) & 0xFF];
            o[5] = table[(v >> 40) & 0xFF];
            o[6] = table[(v >> 48) & 0xFF];
            o[7] = table[v >> 56];
            o += 8;
            pos += 8;
        }
        while (pos < bend) {
            uint64_t v = syn_next(&r);
            for (int j = 0; j < 8 && pos < bend; j++, pos++)
                out[pos - x0] = table[(v >> (8 * j)) & 0xFFu];
        }
        if (sp->n_mode == 1) {
            syn_rng rn = { syn_key(sp->seed, 4, c, blk) };
            double t = sp->n_param * 4294967296.0;
            uint64_t thrn = t >= 4294967296.0 ? 4294967296ULL : (uint64_t)t;
            uint64_t skipn = (x - bstart) / 2;
            rn.s += skipn * SYN_GAMMA;
            uint64_t pn = bstart + skipn * 2;
            while (pn < bend) {
                uint64_t v = syn_next(&rn);
                for (int j = 0; j < 2 && pn < bend; j++, pn++) {
                    uint64_t u = (v >> (32 * j)) & 0xFFFFFFFFULL;
                    if (pn >= x && u < thrn) out[pn - x0] = 'N';
                }
            }
        }
        x = bend;
    }
    if (sp->n_mode == 2 && sp->n_param > 0.0) {
        /* Poisson process of run starts, rate n_param / mean run length per
         * base, generated per block; runs may reach into later blocks */
        double mean_len = 0.5 * ((double)sp->run_min + (double)sp->run_max);
        double lam = sp->n_param / mean_len * (double)SYN_BLOCK;
        uint64_t reach = (sp->run_max + SYN_BLOCK - 1) / SYN_BLOCK;
        uint64_t b_first = x0 / SYN_BLOCK;
        b_first = b_first > reach ? b_first - reach : 0;
        uint64_t b_last = (end - 1) / SYN_BLOCK;
        for (uint64_t b = b_first; b <= b_last; b++) {
            syn_rng r = { syn_key(sp->seed, 5, c, b) };
            /* Poisson(lam) by inversion */
            double u = syn_unif(&r);
            double p = exp(-lam), cdf = p;
            int k = 0;
            while (u > cdf && k < 64) {
                k++;
                p *= lam / k;
                cdf += p;
            }
            for (int i = 0; i < k; i++) {
                uint64_t s = b * SYN_BLOCK + (uint64_t)(syn_unif(&r) * (double)SYN_BLOCK);
                uint64_t len = sp->run_min +
                    (uint64_t)(syn_unif(&r) * (double)(sp->run_max - sp->run_min + 1));
                uint64_t e = s + len;
                if (e > clen) e = clen;
                uint64_t lo = s > x0 ? s : x0, hi = e < end ? e : end;
                for (uint64_t q = lo; q < hi; q++) out[q - x0] = 'N';
            }
        }
    }
}

void synth_fill(uint64_t seed, int n_mode, double n_param, uint32_t run_min, uint32_t run_max,
                uint64_t contig, uint64_t clen, double gc, uint64_t x0, uint64_t n, uint8_t *out)
{
    syn_spec sp = { seed, n_mode, n_param, run_min, run_max };
    fill_range(&sp, contig, clen, gc, x0, n, out);
}

/* multi-threaded fill of many contigs, each written to out + offs[i] */
typedef struct {
    const syn_spec *sp;
    uint64_t first_contig;
    uint64_t n;
    const uint64_t *lens;
    const double *gcs;
    uint8_t *out;
    const uint64_t *offs;
    uint64_t piece;         /* bases per work item */
    uint64_t total_items;
    volatile uint64_t next;  /* shared work counter */
    pthread_mutex_t mu;
    const uint64_t *item_start; /* first work item of each contig (prefix) */
} fill_job;

static void *fill_worker(void *arg)
{
    fill_job *J = (fill_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint64_t it = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (it >= J->total_items) break;
        /* locate contig by binary search on item_start */
        uint64_t lo = 0, hi = J->n;
        while (hi - lo > 1) {
            uint64_t mid = (lo + hi) / 2;
            if (J->item_start[mid] <= it) lo = mid; else hi = mid;
        }
        uint64_t c = lo;
        uint64_t x0 = (it - J->item_start[c]) * J->piece;
        uint64_t n = J->lens[c] - x0;
        if (n > J->piece) n = J->piece;
        fill_range(J->sp, J->first_contig + c, J->lens[c], J->gcs[c], x0, n,
                   J->out + J->offs[c] + x0);
    }
    return NULL;
}

int synth_fill_many(uint64_t seed, int n_mode, double n_param, uint32_t run_min, uint32_t run_max,
                    uint64_t first_contig, uint64_t n, const uint64_t *lens, const double *gcs,
                    uint8_t *out, const uint64_t *offs, int threads)
{
    syn_spec sp = { seed, n_mode, n_param, run_min, run_max };
    fill_job J;
    memset(&J, 0, sizeof J);
    J.sp = &sp;
    J.first_contig = first_contig;
    J.n = n;
    J.lens = lens;
    J.gcs = gcs;
    J.out = out;
    J.offs = offs;
    J.piece = 1ULL << 22;
    uint64_t *is = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    if (!is) return -1;
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        is[i] = acc;
        acc += (lens[i] + J.piece - 1) / J.piece;
    }
    is[n] = acc;
    J.item_start = is;
    J.total_items = acc;
    J.next = 0;
    pthread_mutex_init(&J.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < threads; t++) {
        if (pthread_create(&th[started], NULL, fill_worker, &J) == 0) started++;
    }
    fill_worker(&J);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    free(is);
    return 0;
}

/* ------------------------------------------------------------------ */
/* 2-bit planes: the same bases as fill_range, written as two bit planes  */
/* (for a producer that hands the scan packed data instead of bytes).      */
/* Base x of a chunk is bit x & 31 of word x >> 5; A = (hi 0, lo 0),       */
/* C = (0, 1), G = (1, 1), T = (1, 0). A random byte u gives G/C when its  */
/* low 7 bits are below the GC threshold, and G or T when its top bit is   */
/* set, so hi = the top bit and lo = (u & 0x7F) < thr.                     */
/* ------------------------------------------------------------------ */

/* OR the low cnt (<= 32) bits of v into bits [p, p + cnt) of a plane */
static inline void put_bits(uint32_t *pl, uint64_t p, uint32_t v, uint32_t cnt)
{
    if (cnt < 32) v &= (1u << cnt) - 1u;
    const uint64_t w = p >> 5;
    const uint32_t sh = (uint32_t)(p & 31);
    pl[w] |= v << sh;
    if (sh && cnt > 32 - sh) pl[w + 1] |= v >> (32 - sh);
}

#if defined(__x86_64__)
/* 4 draws from state s (not advanced): the hi / lo bits of their 32 bases */
__attribute__((target("avx2"))) static inline void draws4_bits(uint64_t s, uint32_t thr,
                                                               uint32_t *hb, uint32_t *lb)
{
    const __m256i g = _mm256_set_epi64x((long long)(4 * SYN_GAMMA), (long long)(3 * SYN_GAMMA),
                                        (long long)(2 * SYN_GAMMA), (long long)SYN_GAMMA);
    __m256i z = _mm256_add_epi64(_mm256_set1_epi64x((long long)s), g);
    z = syn_mul64(_mm256_xor_si256(z, _mm256_srli_epi64(z, 30)), 0xBF58476D1CE4E5B9ULL);
    z = syn_mul64(_mm256_xor_si256(z, _mm256_srli_epi64(z, 27)), 0x94D049BB133111EBULL);
    z = _mm256_xor_si256(z, _mm256_srli_epi64(z, 31));
    const __m256i low7 = _mm256_and_si256(z, _mm256_set1_epi8(0x7F));
    const __m256i at = _mm256_cmpeq_epi8(_mm256_max_epu8(low7, _mm256_set1_epi8((char)thr)), low7);
    *hb = (uint32_t)_mm256_movemask_epi8(z);
    *lb = ~(uint32_t)_mm256_movemask_epi8(at);
}
#endif

/* bases [x0, x0 + n) of contig c (length clen, GC gc), whose base 0 is base
 * cstart of the chunk, into the chunk planes (bits ORed in; n_mode 0 only) */
static void pack_range(const syn_spec *sp, uint64_t c, uint64_t clen, double gc, uint64_t cstart,
                       uint64_t x0, uint64_t n, uint32_t *hi, uint32_t *lo)
{
    if (x0 >= clen) return;
    if (x0 + n > clen) n = clen - x0;
    const uint32_t thr = (uint32_t)(gc * 128.0 + 0.5);
    uint64_t x = x0, end = x0 + n;
    while (x < end) {
        const uint64_t blk = x / SYN_BLOCK;
        const uint64_t bstart = blk * SYN_BLOCK;
        const uint64_t bend = bstart + SYN_BLOCK < end ? bstart + SYN_BLOCK : end;
        syn_rng r = { syn_key(sp->seed, 3, c, blk) };
        const uint64_t skip = (x - bstart) / 8;
        r.s += skip * SYN_GAMMA;
        uint64_t pos = bstart + skip * 8;
        while (pos < bend) {
#if defined(__x86_64__)
            if (syn_simd && pos >= x && pos + 32 <= bend && __builtin_cpu_supports("avx2")) {
                uint32_t hb, lb;
                draws4_bits(r.s, thr, &hb, &lb);
                r.s += 4 * SYN_GAMMA;
                put_bits(hi, cstart + pos, hb, 32);
                put_bits(lo, cstart + pos, lb, 32);
                pos += 32;
                continue;
            }
#endif
            const uint64_t v = syn_next(&r);
            uint32_t hb = 0, lb = 0;
            for (uint32_t j = 0; j < 8; j++) {
                const uint32_t u = (uint32_t)(v >> (8 * j)) & 0xFFu;
                hb |= (u >> 7) << j;
                lb |= ((u & 0x7Fu) < thr ? 1u : 0u) << j;
            }
            const uint64_t a = pos > x ? pos : x, b = pos + 8 < bend ? pos + 8 : bend;
            put_bits(hi, cstart + a, hb >> (a - pos), (uint32_t)(b - a));
            put_bits(lo, cstart + a, lb >> (a - pos), (uint32_t)(b - a));
            pos += 8;
        }
        x = bend;
    }
}

typedef struct {
    const syn_spec *sp;
    uint64_t first_contig, n;
    const uint64_t *lens, *starts;   /* starts: chunk offset of each contig (prefix sums) */
    const double *gcs;
    uint32_t *hi, *lo;
    uint64_t words, item_words, items;
    volatile uint64_t next;
    pthread_mutex_t mu;
} pack_job;

static void *pack_worker(void *arg)
{
    pack_job *J = (pack_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->mu);
        const uint64_t it = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (it >= J->items) break;
        const uint64_t w0 = it * J->item_words;
        const uint64_t w1 = w0 + J->item_words < J->words ? w0 + J->item_words : J->words;
        memset(J->hi + w0, 0, (w1 - w0) * sizeof(uint32_t));
        memset(J->lo + w0, 0, (w1 - w0) * sizeof(uint32_t));
        const uint64_t b0 = 32 * w0, b1 = 32 * w1;
        /* first contig ending after b0 */
        uint64_t lo_i = 0, hi_i = J->n;
        while (lo_i < hi_i) {
            const uint64_t mid = (lo_i + hi_i) / 2;
            if (J->starts[mid] + J->lens[mid] <= b0) lo_i = mid + 1; else hi_i = mid;
        }
        for (uint64_t i = lo_i; i < J->n && J->starts[i] < b1; i++) {
            const uint64_t cs = J->starts[i], ce = cs + J->lens[i];
            const uint64_t a = cs > b0 ? cs : b0, b = ce < b1 ? ce : b1;
            if (a < b)
                pack_range(J->sp, J->first_contig + i, J->lens[i], J->gcs[i], cs, a - cs, b - a,
                           J->hi, J->lo);
        }
    }
    return NULL;
}

/* hi / lo planes (ceil(total / 32) words each, written whole; bits past the
 * last base 0) of contigs first_contig .. first_contig + n - 1 packed back
 * to back from base 0. Only references without N (n_mode 0). */
int synth_fill_packed(uint64_t seed, uint64_t first_contig, uint64_t n, const uint64_t *lens,
                      const double *gcs, uint32_t *hi, uint32_t *lo, int threads)
{
    syn_spec sp = { seed, 0, 0.0, 0, 0 };
    uint64_t *starts = (uint64_t *)malloc((n + 1) * sizeof(uint64_t));
    if (!starts) return -1;
    uint64_t acc = 0;
    for (uint64_t i = 0; i < n; i++) {
        starts[i] = acc;
        acc += lens[i];
    }
    starts[n] = acc;
    pack_job J;
    memset(&J, 0, sizeof J);
    J.sp = &sp;
    J.first_contig = first_contig;
    J.n = n;
    J.lens = lens;
    J.starts = starts;
    J.gcs = gcs;
    J.hi = hi;
    J.lo = lo;
    J.words = (acc + 31) / 32;
    J.item_words = 1ULL << 16;
    J.items = (J.words + J.item_words - 1) / J.item_words;
    pthread_mutex_init(&J.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < threads; t++)
        if (pthread_create(&th[started], NULL, pack_worker, &J) == 0) started++;
    pack_worker(&J);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.mu);
    free(starts);
    return 0;
}

/* ------------------------------------------------------------------ */
/* queries                                                             */
/* ------------------------------------------------------------------ */

/*
 * n queries, lengths uniform in [lmin, lmax], bases iid uniform ACGT.
 * Query i is written to out + i * stride (stride >= lmax); lens[i] = length.
 */
void synth_queries(uint64_t seed, uint64_t stream_tag, uint64_t n, uint32_t lmin, uint32_t lmax,
                   uint8_t *out, uint64_t stride, uint32_t *lens)
{
    static const uint8_t acgt[4] = { 'A', 'C', 'G', 'T' };
    for (uint64_t i = 0; i < n; i++) {
        syn_rng r = { syn_key(seed, 6, stream_tag, i) };
        uint32_t L = lmin + (uint32_t)(syn_unif(&r) * (double)(lmax - lmin + 1));
        if (L > lmax) L = lmax;
        lens[i] = L;
        uint8_t *q = out + i * stride;
        uint64_t v = 0;
        for (uint32_t j = 0; j < L; j++) {
            if ((j & 31) == 0) v = syn_next(&r);
            q[j] = acgt[(v >> (2 * (j & 31))) & 3];
        }
    }
}
