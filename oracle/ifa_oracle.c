/*
 * ifa_oracle.c -- plain CPU oracle for the brute-force gapless scan.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library. The product path
 * never calls it, and it shares no code, header or table with the HIP path.
 *
 * What it computes is the plain definition of the paper's brute-force mode
 * (Methods, "Algorithm Design": every start position is tested and every valid
 * alignment is reported; the distance is Hamming, substitutions only, with a
 * user threshold up to the full query length -- Abstract and Introduction).
 * Readings taken where the paper is silent:
 *   - both strands: the minus strand compares the reverse complement of the
 *     query against the forward reference window; pos is the 0-based
 *     leftmost forward coordinate in the contig;
 *   - reference non-ACGT bytes (N) are counted apart from substitutions, in
 *     n_ref, with their own threshold maxN (Methods, "Algorithm Design" and
 *     "SIMD Optimization": Ns tracked separately, per-lane substitution and
 *     clip counts); default maxN = floor(L/4) after the 25% soft-clip default;
 *   - bytes are case-insensitive; every byte other than ACGT/acgt is N;
 *   - a query N against a reference A/C/G/T is a substitution; a query N
 *     against a reference N counts only in n_ref;
 *   - a window is a hit iff m <= K and n_ref <= M ("exceed" ends a lane in
 *     the SIMD kernel description, so equality is still a hit), with
 *     K = min(maxSubs, L) and M = min(maxN, L);
 *   - without overhang only windows wholly inside one contig are tested;
 *   - policy AS_MISMATCH (alternative reading): every reference or query N
 *     position counts in m and there is no maxN test.
 * Overhang (Methods, "Algorithm Design": soft-clipped alignments at contig
 * boundaries, up to 25% of the query length by default; short contigs are
 * fused with N padding and the kernel counts reference Ns apart from
 * substitutions). Readings:
 *   - a window may start at p in [-C, n - L + C]; its bases off the contig
 *     read as N, so they count in n_ref (and, under AS_MISMATCH, in m);
 *   - the clip limit is C = min(maxN, L - 1) with the same maxN (default
 *     floor(L/4)): the paper's clip count is its reference-N count, and a
 *     window keeps at least one base on the contig;
 *   - the off-contig bases of a window, left and right together, must not
 *     exceed C (under N_SEPARATE n_ref <= M implies it);
 *   - pos is the window's first base, negative for a left overhang;
 *   - a contig is never fused with its neighbour: off-contig bases are N
 *     whatever lies beyond the contig in the input.
 * Output order is reference order (Results, "Accuracy Validation": the
 * primary is the first valid alignment in reference order), tie-broken by
 * strand (+ first) then query index.
 *
 * Indexed mode (Methods, "Algorithm Design"): query k-mer seeds, a central
 * portion of each k-mer optionally masked, sampled every `step` offsets; a
 * window is reported only if it is a hit as above AND at least T of the
 * query's valid seeds (no N at an unmasked position) occur error-free at the
 * same offset of the window (reference bases equal at every unmasked
 * position). T comes from the MinHits computation below (orc_minhits) and the
 * k from the longest-k rule; those choices are made by the caller and passed
 * in (orc_seed_spec). Overhanging windows are not combined with seeds.
 *
 * Count+digest: per query, the number of hits and the wrapping 64-bit sum of
 *   H = mix64(((contig << 32) | pos) ^ (aux << 45)),
 *   aux = strand | (mismatches << 1) | (n_ref << 10),
 * where mix64 is the SplitMix64 output finaliser (Steele, Lea & Flood 2014).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef struct {
    uint32_t query;
    uint32_t contig;
    int32_t pos;
    uint8_t strand;
    uint8_t n_ref;
    uint16_t mismatches;
} orc_hit;

enum { ORC_N_SEPARATE = 0, ORC_N_AS_MISMATCH = 1 };

/* Indexed-mode seeds: k[j] per query, thr[2j + s] per query strand, the
 * length of the masked centre of every k-mer, and the sampling step. */
typedef struct {
    const int32_t *k;
    const int32_t *thr;
    int32_t mask;
    int32_t step;
} orc_seed_spec;

/* base code: A 0, C 1, G 2, T 3, anything else 4 (N) */
static int orc_norm(uint8_t b)
{
    switch (b) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return 4;
    }
}

static int orc_comp(int x)
{
    return x < 4 ? 3 - x : 4;
}

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* pos enters the key as its 32-bit two's complement pattern */
uint64_t orc_hit_hash(uint32_t contig, int32_t pos, uint32_t strand, uint32_t mism,
                      uint32_t nref)
{
    uint64_t key = ((uint64_t)contig << 32) | (uint64_t)(uint32_t)pos;
    uint64_t aux = (uint64_t)strand | ((uint64_t)mism << 1) | ((uint64_t)nref << 10);
    return orc_mix64(key ^ (aux << 45));
}

/* ------------------------------------------------------------------ */

typedef struct {
    int L;
    int K;              /* min(maxSubs, L) */
    int M;              /* min(maxN, L) */
    int C;              /* clip limit min(maxN, L - 1); used with overhang */
    uint8_t *code[2];   /* [0] query codes, [1] reverse complement */
} orc_query;

typedef struct {
    uint32_t contig;    /* index into the contig arrays */
    uint64_t p0, p1;    /* window starts [p0, p1) inside the contig */
    int edge;           /* 1: instead, the overhanging windows of the contig */
} orc_item;

typedef struct {
    /* inputs */
    uint32_t nq;
    orc_query *qs;
    const uint8_t *const *ctg;
    const uint64_t *clen;
    uint32_t first_ordinal;
    uint32_t strands;
    uint32_t policy;
    int overhang;
    const orc_seed_spec *seeds;   /* NULL: brute force, no seed condition */
    int want_records;
    int maxL;
    orc_item *items;
    uint64_t n_items;
    /* shared cursor */
    uint64_t next;
    pthread_mutex_t mu;
    int failed;
} orc_job;

typedef struct {
    orc_job *J;
    orc_hit *hits;
    uint64_t n, cap;
    uint64_t *counts;
    uint64_t *digests;
    int failed;
} orc_worker;

static int push_hit(orc_worker *W, const orc_hit *h)
{
    if (W->n == W->cap) {
        uint64_t nc = W->cap ? W->cap * 2 : 1024;
        orc_hit *p = (orc_hit *)realloc(W->hits, nc * sizeof(orc_hit));
        if (!p) return -1;
        W->hits = p;
        W->cap = nc;
    }
    W->hits[W->n++] = *h;
    return 0;
}

/* Test one window: mismatches m and reference-N count nref for query code
 * array qc of length L against reference codes r[0..L). Returns 1 on a hit.
 * The mismatch loop may stop once m exceeds K; that cannot change the hit
 * decision, and m is reported only for hits. */
static int orc_test_window(const uint8_t *qc, int L, const uint8_t *r, int K, int M,
                           uint32_t policy, int *m_out, int *nref_out)
{
    int m = 0;
    if (policy == ORC_N_SEPARATE) {
        for (int i = 0; i < L; i++) {
            if (r[i] != 4 && qc[i] != r[i]) {
                m++;
                if (m > K) return 0;
            }
        }
    } else {
        for (int i = 0; i < L; i++) {
            if (r[i] == 4 || qc[i] == 4 || qc[i] != r[i]) {
                m++;
                if (m > K) return 0;
            }
        }
    }
    int nref = 0;
    for (int i = 0; i < L; i++)
        if (r[i] == 4) nref++;
    if (policy == ORC_N_SEPARATE && nref > M) return 0;
    *m_out = m;
    *nref_out = nref;
    return 1;
}

/* Error-free seeds of query strand codes qc (length L) in the window r: the
 * sampled offsets i = 0, step, 2 step, ... (i + k <= L) whose k-mer holds no
 * query N at an unmasked position and equals the window's bases at every
 * unmasked position. The masked centre is [(k - mask) / 2, that + mask). */
static int orc_seed_hits(const uint8_t *qc, int L, const uint8_t *r, int k, int mask, int step)
{
    const int lo = (k - mask) / 2, hi = lo + mask;
    int hits = 0;
    for (int i = 0; i + k <= L; i += step) {
        int valid = 1, match = 1;
        for (int t = 0; t < k; t++) {
            if (t >= lo && t < hi) continue;
            if (qc[i + t] == 4) {
                valid = 0;
                break;
            }
            if (r[i + t] != qc[i + t]) match = 0;   /* a reference N equals nothing */
        }
        hits += valid && match;
    }
    return hits;
}

/* The seed condition of indexed mode (always true without seeds). */
static int orc_seeds_ok(const orc_job *J, uint32_t j, int s, const uint8_t *qc, int L,
                        const uint8_t *r)
{
    if (!J->seeds) return 1;
    const orc_seed_spec *S = J->seeds;
    return orc_seed_hits(qc, L, r, S->k[j], S->mask, S->step) >= S->thr[2 * j + s];
}

static void emit_hit(orc_worker *W, uint32_t j, uint32_t contig, int64_t p, int s, int m,
                     int nref)
{
    orc_job *J = W->J;
    orc_hit h;
    h.query = j;
    h.contig = J->first_ordinal + contig;
    h.pos = (int32_t)p;
    h.strand = (uint8_t)s;
    h.n_ref = (uint8_t)nref;
    h.mismatches = (uint16_t)m;
    if (W->counts) W->counts[j] += 1;
    if (W->digests)
        W->digests[j] += orc_hit_hash(h.contig, h.pos, h.strand, h.mismatches, h.n_ref);
    if (J->want_records && push_hit(W, &h) != 0) W->failed = 1;
}

/* The overhanging windows of one contig: starts p in [-C, n - L + C] that
 * are not wholly inside it, with at most C bases off the contig, which read
 * as N. */
static void run_edge(orc_worker *W, uint32_t contig, uint8_t *win)
{
    orc_job *J = W->J;
    const uint8_t *src = J->ctg[contig];
    const int64_t n = (int64_t)J->clen[contig];
    for (uint32_t j = 0; j < J->nq; j++) {
        const orc_query *Q = &J->qs[j];
        const int64_t L = Q->L, C = Q->C;
        for (int64_t p = -C; p <= n - L + C; p++) {
            if (p >= 0 && p <= n - L) {                    /* wholly inside: skip them */
                p = n - L;
                continue;
            }
            int64_t off = 0;
            for (int64_t i = 0; i < L; i++) {
                const int64_t x = p + i;
                if (x < 0 || x >= n) {
                    win[i] = 4;
                    off++;
                } else {
                    win[i] = (uint8_t)orc_norm(src[x]);
                }
            }
            if (off > C) continue;
            for (int s = 0; s < 2; s++) {
                if (!(J->strands & (1u << s))) continue;
                int m, nref;
                if (!orc_test_window(Q->code[s], (int)L, win, Q->K, Q->M, J->policy, &m,
                                     &nref))
                    continue;
                emit_hit(W, j, contig, p, s, m, nref);
                if (W->failed) return;
            }
        }
    }
}

static void run_item(orc_worker *W, const orc_item *it, uint8_t *codes)
{
    orc_job *J = W->J;
    if (it->edge) {
        run_edge(W, it->contig, codes);
        return;
    }
    const uint8_t *src = J->ctg[it->contig];
    uint64_t n = J->clen[it->contig];
    /* normalise the bases this item's windows can touch */
    uint64_t a = it->p0;
    uint64_t b = it->p1 + (uint64_t)J->maxL;
    if (b > n) b = n;
    for (uint64_t x = a; x < b; x++) codes[x - a] = (uint8_t)orc_norm(src[x]);
    for (uint32_t j = 0; j < J->nq; j++) {
        const orc_query *Q = &J->qs[j];
        int L = Q->L;
        if ((uint64_t)L > n) continue;
        uint64_t last = n - (uint64_t)L;      /* last valid start */
        uint64_t pe = it->p1;
        if (pe > last + 1) pe = last + 1;
        for (uint64_t p = it->p0; p < pe; p++) {
            const uint8_t *r = codes + (p - a);
            for (int s = 0; s < 2; s++) {
                if (!(J->strands & (1u << s))) continue;
                int m, nref;
                if (!orc_test_window(Q->code[s], L, r, Q->K, Q->M, J->policy, &m, &nref))
                    continue;
                if (!orc_seeds_ok(J, j, s, Q->code[s], L, r)) continue;
                emit_hit(W, j, it->contig, (int64_t)p, s, m, nref);
                if (W->failed) return;
            }
        }
    }
}

#define ORC_ITEM_WINDOWS (1u << 20)

static void *orc_worker_main(void *arg)
{
    orc_worker *W = (orc_worker *)arg;
    orc_job *J = W->J;
    /* also the window buffer of edge items (maxL codes) */
    uint8_t *codes = (uint8_t *)malloc(ORC_ITEM_WINDOWS + (size_t)J->maxL + 1);
    if (!codes) {
        W->failed = 1;
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&J->mu);
        uint64_t i = J->next++;
        pthread_mutex_unlock(&J->mu);
        if (i >= J->n_items) break;
        run_item(W, &J->items[i], codes);
        if (W->failed) break;
    }
    free(codes);
    return NULL;
}

static int hit_cmp(const void *x, const void *y)
{
    const orc_hit *a = (const orc_hit *)x, *b = (const orc_hit *)y;
    if (a->contig != b->contig) return a->contig < b->contig ? -1 : 1;   /* pos is signed */
    if (a->pos != b->pos) return a->pos < b->pos ? -1 : 1;
    if (a->strand != b->strand) return a->strand < b->strand ? -1 : 1;
    if (a->query != b->query) return a->query < b->query ? -1 : 1;
    return 0;
}

void orc_free(void *p)
{
    free(p);
}

/*
 * Scan every query against every contig. Returns 0 on success, -1 on bad
 * arguments or allocation failure. When want_records is set, *out receives a
 * malloc'd array of *n_out hits in (contig, pos, strand, query) order (free
 * with orc_free). counts/digests, when not NULL, are nq-long arrays that this
 * call overwrites. overhang = 1 adds the windows that hang off a contig end;
 * seeds (may be NULL) adds the indexed-mode seed condition.
 * Contigs must be shorter than 2^31 bases (pos is an int32).
 */
int orc_scan(uint32_t nq, const uint8_t *const *q, const uint32_t *qlen,
             const int32_t *max_subs, const int32_t *max_n,
             uint32_t nc, const uint8_t *const *ctg, const uint64_t *clen,
             uint32_t first_ordinal, uint32_t strands, uint32_t policy, int overhang,
             const orc_seed_spec *seeds, int threads, int want_records, orc_hit **out,
             uint64_t *n_out, uint64_t *counts, uint64_t *digests)
{
    if (out) *out = NULL;
    if (n_out) *n_out = 0;
    if (strands < 1 || strands > 3 || policy > 1 || overhang < 0 || overhang > 1) return -1;
    if (seeds && (overhang || !seeds->k || !seeds->thr || seeds->step < 1 || seeds->mask < 0))
        return -1;
    for (uint32_t c = 0; c < nc; c++)
        if (clen[c] >= (1ull << 31)) return -1;
    orc_job J;
    memset(&J, 0, sizeof J);
    J.nq = nq;
    J.ctg = ctg;
    J.clen = clen;
    J.first_ordinal = first_ordinal;
    J.strands = strands;
    J.policy = policy;
    J.overhang = overhang;
    J.seeds = seeds;
    J.want_records = want_records;
    J.qs = (orc_query *)calloc(nq ? nq : 1, sizeof(orc_query));
    if (!J.qs) return -1;
    int rc = -1;
    J.maxL = 1;
    for (uint32_t j = 0; j < nq; j++) {
        int L = (int)qlen[j];
        if (L < 1 || max_subs[j] < 0 || (max_n && max_n[j] < 0)) goto done;
        if (seeds && (seeds->k[j] < 1 || seeds->k[j] > L || seeds->mask >= seeds->k[j]))
            goto done;
        orc_query *Q = &J.qs[j];
        Q->L = L;
        Q->K = max_subs[j] < L ? max_subs[j] : L;
        int mn = max_n ? max_n[j] : L / 4;
        Q->M = mn < L ? mn : L;
        Q->C = mn < L - 1 ? mn : L - 1;
        Q->code[0] = (uint8_t *)malloc((size_t)L);
        Q->code[1] = (uint8_t *)malloc((size_t)L);
        if (!Q->code[0] || !Q->code[1]) goto done;
        for (int i = 0; i < L; i++) Q->code[0][i] = (uint8_t)orc_norm(q[j][i]);
        for (int i = 0; i < L; i++) Q->code[1][i] = (uint8_t)orc_comp(Q->code[0][L - 1 - i]);
        if (L > J.maxL) J.maxL = L;
    }
    /* work items: ranges of window starts, small enough that every thread
     * gets several even when there is one contig */
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    uint64_t total_bases = 0;
    for (uint32_t c = 0; c < nc; c++) total_bases += clen[c];
    uint64_t item = total_bases / ((uint64_t)threads * 8u);
    if (item < 4096) item = 4096;
    if (item > ORC_ITEM_WINDOWS) item = ORC_ITEM_WINDOWS;
    uint64_t n_items = overhang ? nc : 0;
    for (uint32_t c = 0; c < nc; c++)
        n_items += (clen[c] + item - 1) / item;
    J.items = (orc_item *)malloc((n_items ? n_items : 1) * sizeof(orc_item));
    if (!J.items) goto done;
    J.n_items = 0;
    for (uint32_t c = 0; c < nc; c++) {
        for (uint64_t p = 0; p < clen[c]; p += item) {
            orc_item *it = &J.items[J.n_items++];
            it->contig = c;
            it->p0 = p;
            it->p1 = p + item < clen[c] ? p + item : clen[c];
            it->edge = 0;
        }
        if (overhang) {
            orc_item *it = &J.items[J.n_items++];
            it->contig = c;
            it->p0 = it->p1 = 0;
            it->edge = 1;
        }
    }
    pthread_mutex_init(&J.mu, NULL);
    orc_worker *W = (orc_worker *)calloc((size_t)threads, sizeof(orc_worker));
    pthread_t *th = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    int *started = (int *)calloc((size_t)threads, sizeof(int));
    if (!W || !th || !started) {
        free(W);
        free(th);
        free(started);
        pthread_mutex_destroy(&J.mu);
        goto done;
    }
    int alloc_fail = 0;
    for (int t = 0; t < threads; t++) {
        W[t].J = &J;
        if (counts) W[t].counts = (uint64_t *)calloc(nq ? nq : 1, sizeof(uint64_t));
        if (digests) W[t].digests = (uint64_t *)calloc(nq ? nq : 1, sizeof(uint64_t));
        if ((counts && !W[t].counts) || (digests && !W[t].digests)) alloc_fail = 1;
    }
    if (!alloc_fail) {
        for (int t = 1; t < threads; t++)
            started[t] = pthread_create(&th[t], NULL, orc_worker_main, &W[t]) == 0;
        orc_worker_main(&W[0]);
        for (int t = 1; t < threads; t++)
            if (started[t]) pthread_join(th[t], NULL);
    }
    int failed = alloc_fail;
    uint64_t total = 0;
    for (int t = 0; t < threads; t++) {
        failed |= W[t].failed;
        total += W[t].n;
    }
    if (!failed) {
        if (counts) memset(counts, 0, (size_t)nq * sizeof(uint64_t));
        if (digests) memset(digests, 0, (size_t)nq * sizeof(uint64_t));
        for (int t = 0; t < threads; t++)
            for (uint32_t j = 0; j < nq; j++) {
                if (counts) counts[j] += W[t].counts[j];
                if (digests) digests[j] += W[t].digests[j];
            }
        if (want_records) {
            orc_hit *all = (orc_hit *)malloc((total ? total : 1) * sizeof(orc_hit));
            if (!all) {
                failed = 1;
            } else {
                uint64_t k = 0;
                for (int t = 0; t < threads; t++) {
                    if (W[t].n) memcpy(all + k, W[t].hits, W[t].n * sizeof(orc_hit));
                    k += W[t].n;
                }
                qsort(all, total, sizeof(orc_hit), hit_cmp);
                if (out) *out = all; else free(all);
                if (n_out) *n_out = total;
            }
        }
    }
    for (int t = 0; t < threads; t++) {
        free(W[t].hits);
        free(W[t].counts);
        free(W[t].digests);
    }
    free(W);
    free(th);
    free(started);
    pthread_mutex_destroy(&J.mu);
    rc = failed ? -1 : 0;
done:
    for (uint32_t j = 0; j < nq; j++) {
        free(J.qs[j].code[0]);
        free(J.qs[j].code[1]);
    }
    free(J.qs);
    free(J.items);
    return rc;
}

/*
 * Evaluate one (query, window, strand) exactly, without the early stop:
 * writes the full mismatch count and n_ref. Returns 1 if the window is a hit,
 * 0 if not, -1 if it is not a window of the scan (it leaves the contig, or,
 * with overhang, leaves it by more than the clip limit) or arguments are bad.
 */
int orc_eval_window(const uint8_t *q, uint32_t L, int32_t max_subs, int32_t max_n,
                    const uint8_t *ctg, uint64_t clen, int64_t pos, uint32_t strand,
                    uint32_t policy, int overhang, int32_t *m_out, int32_t *nref_out)
{
    if (L < 1 || strand > 1 || max_subs < 0 || policy > 1 || clen >= (1ull << 31))
        return -1;
    int K = max_subs < (int32_t)L ? max_subs : (int32_t)L;
    int mn = max_n < 0 ? (int)L / 4 : max_n;
    int M = mn < (int)L ? mn : (int)L;
    int C = mn < (int)L - 1 ? mn : (int)L - 1;
    const int64_t n = (int64_t)clen;
    int off = 0;
    for (uint32_t i = 0; i < L; i++)
        if (pos + (int64_t)i < 0 || pos + (int64_t)i >= n) off++;
    if (overhang ? off > C : off > 0) return -1;
    int m = 0, nref = 0;
    for (uint32_t i = 0; i < L; i++) {
        int qc = strand == 0 ? orc_norm(q[i]) : orc_comp(orc_norm(q[L - 1 - i]));
        const int64_t x = pos + (int64_t)i;
        int r = (x < 0 || x >= n) ? 4 : orc_norm(ctg[x]);
        if (r == 4) nref++;
        if (policy == ORC_N_SEPARATE) {
            if (r != 4 && qc != r) m++;
        } else {
            if (r == 4 || qc == 4 || qc != r) m++;
        }
    }
    *m_out = m;
    *nref_out = nref;
    if (m > K) return 0;
    if (policy == ORC_N_SEPARATE && nref > M) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* MinHits (Methods, "Algorithm Design"): the minimum number of error-free
 * seeds that a valid alignment keeps with a given probability, by Monte
 * Carlo with a fixed seed; at probability 1 the deterministic lower bound
 * validKmers - kEffective * maxSubs - maxClips.
 *
 * Model (readings): a query with V valid seeds is taken as V k-mers at
 * offsets 0, step, ..., (V - 1) step over a span of (V - 1) step + k bases
 * (for an N-free query sampled every base, exactly its L bases); each trial
 * places min(maxSubs, span) substitutions at distinct positions drawn
 * uniformly over the span, and counts the seeds with no substitution at an
 * unmasked position. The answer is the largest t with at least ppm / 10^6 of
 * the trials keeping t or more seeds. kEffective is the most seeds one
 * substitution can touch; maxClips is 0 (seeds are not combined with
 * overhanging windows).
 *
 * Random draws: SplitMix64 (Steele, Lea & Flood 2014), draw n of stream
 * `seed` = mix64(seed + (n + 1) * 0x9E3779B97F4A7C15); a uniform position in
 * [0, m) is the high 64 bits of draw * m (Lemire's multiply-shift). A trial
 * picks its positions by a partial Fisher-Yates shuffle (slot c swapped with
 * a uniform slot in [c, span)) of the position array the previous trial left
 * (initially 0, 1, ..., span - 1); the draw counter runs on across trials.
 */
uint64_t orc_splitmix64(uint64_t seed, uint64_t n)
{
    return orc_mix64(seed + (n + 1) * 0x9E3779B97F4A7C15ULL);
}

static int orc_kmer_unmasked(int t, int k, int mask)
{
    const int lo = (k - mask) / 2;
    return t < lo || t >= lo + mask;
}

int orc_keff(int k, int mask, int step)
{
    int best = 0;
    for (int x = 0; x < k + step * k; x++) {
        int c = 0;
        for (int v = 0; v * step <= x; v++) {
            const int t = x - v * step;
            if (t < k && orc_kmer_unmasked(t, k, mask)) c++;
        }
        if (c > best) best = c;
    }
    return best;
}

/* MinHits; may be <= 0 (the caller takes max(1, .)). INT64_MIN on bad
 * arguments or no memory. */
int64_t orc_minhits(int32_t V, int32_t subs, int32_t k, int32_t mask, int32_t step,
                    uint64_t iters, uint64_t seed, uint32_t ppm)
{
    if (V <= 0 || k < 1 || mask < 0 || mask >= k || step < 1 || subs < 0 || ppm > 1000000)
        return INT64_MIN;
    const int span = (V - 1) * step + k;
    const int s = subs < span ? subs : span;
    if (ppm == 1000000) return (int64_t)V - (int64_t)orc_keff(k, mask, step) * s;
    if (iters == 0) return INT64_MIN;
    int *pos = (int *)malloc((size_t)span * sizeof(int));
    uint8_t *dead = (uint8_t *)malloc((size_t)V);
    uint64_t *hist = (uint64_t *)calloc((size_t)V + 1, sizeof(uint64_t));
    if (!pos || !dead || !hist) {
        free(pos);
        free(dead);
        free(hist);
        return INT64_MIN;
    }
    for (int i = 0; i < span; i++) pos[i] = i;
    uint64_t n = 0;
    for (uint64_t it = 0; it < iters; it++) {
        for (int c = 0; c < s; c++) {
            const uint64_t r = orc_splitmix64(seed, n++);
            const int j = c + (int)(((unsigned __int128)r * (uint64_t)(span - c)) >> 64);
            const int tmp = pos[c];
            pos[c] = pos[j];
            pos[j] = tmp;
        }
        memset(dead, 0, (size_t)V);
        for (int c = 0; c < s; c++) {
            const int x = pos[c];
            for (int v = 0; v < V; v++) {
                const int t = x - v * step;
                if (t >= 0 && t < k && orc_kmer_unmasked(t, k, mask)) dead[v] = 1;
            }
        }
        int alive = 0;
        for (int v = 0; v < V; v++) alive += !dead[v];
        hist[alive]++;
    }
    int64_t ans = 0;
    uint64_t acc = 0;
    for (int t = V; t >= 0; t--) {
        acc += hist[t];
        if ((unsigned __int128)acc * 1000000u >= (unsigned __int128)ppm * iters) {
            ans = t;
            break;
        }
    }
    free(pos);
    free(dead);
    free(hist);
    return ans;
}
