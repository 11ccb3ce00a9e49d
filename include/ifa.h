/*
 * ifa.h -- C ABI of libifa.so, the MI355X (gfx950) brute-force gapless scan.
 *
 * The library implements the brute-force mode of IndelFreeAligner (Methods,
 * "Algorithm Design"): every query is tested, forward and reverse complement,
 * against every start position of a reference that is streamed in contig by
 * contig, and every window whose Hamming distance is at most the query's
 * threshold is reported. Thresholds may go up to the full query length
 * (Abstract; "Mismatch Tolerance Scalability"). Reference Ns are counted apart
 * from substitutions (Methods, "Algorithm Design"; "SIMD Optimization").
 * Device memory does not grow with the total reference size (Methods,
 * "Memory Management").
 *
 * Definition computed for query j (length L, threshold k, N threshold maxN),
 * strand s and every window [p, p + L) lying wholly inside one contig:
 *   n_ref = number of window positions holding a reference non-ACGT byte;
 *   IFA_N_SEPARATE (default):
 *     m   = positions where the reference base is A/C/G/T and differs from
 *           the query base (a query non-ACGT byte differs from every A/C/G/T);
 *     hit iff m <= min(k, L) and n_ref <= min(maxN, L);
 *   IFA_N_AS_MISMATCH:
 *     m   = positions where either side is non-ACGT or the bases differ;
 *     hit iff m <= min(k, L).
 * Strand 0 compares the query itself, strand 1 its reverse complement, both
 * against the forward reference; pos is the 0-based leftmost forward
 * coordinate of the window in its contig. Bytes are case-insensitive; every
 * byte other than A/C/G/T/a/c/g/t is N.
 *
 * With IFA_FLAG_OVERHANG (soft-clipped alignments at contig boundaries,
 * Methods, "Algorithm Design": up to 25 % of the query length by default;
 * short contigs are fused with N padding) the windows also include those that
 * hang off either end of a contig, or both: starts p in [-C, n - L + C] for a
 * contig of n bases, C = min(maxN, L - 1), with at most C of the window's
 * bases off the contig. Off-contig bases read as N in the definition above
 * (they count in n_ref, and in m under IFA_N_AS_MISMATCH). pos is then
 * negative for a window that hangs off the left end. A contig is never
 * fused with its neighbour.
 *
 * General conventions
 *   - Every entry point returns an ifa_status; a failed call changes nothing
 *     (all or nothing) and leaves a message for ifa_last_error.
 *   - Input buffers belong to the caller and may be reused as soon as the
 *     call returns: the library packs what it needs into its own pinned host
 *     memory before returning. Output arrays belong to the caller. The
 *     context, its device memory and its pinned memory belong to the library.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - All pointers in this header are host pointers.
 */
#ifndef IFA_H
#define IFA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IFA_ABI_VERSION 4u
/* Longest query: n_ref and the mismatch count of a window then fit the
 * record's fields (n_ref is one byte). */
#define IFA_MAX_QUERY_LEN 255u

typedef struct ifa_ctx ifa_ctx;

typedef enum {
    IFA_OK = 0,
    IFA_E_INVALID = 1,   /* bad argument */
    IFA_E_NOMEM = 2,     /* host or device allocation failed */
    IFA_E_DEVICE = 3,    /* HIP runtime error */
    IFA_E_STATE = 4,     /* call not allowed in the context's current state */
    IFA_E_TOO_LONG = 5   /* query longer than IFA_MAX_QUERY_LEN, or empty */
} ifa_status;

enum { IFA_N_SEPARATE = 0, IFA_N_AS_MISMATCH = 1 };
enum { IFA_SINK_RECORDS = 0, IFA_SINK_COUNT_DIGEST = 1 };
enum { IFA_STRAND_FWD = 1, IFA_STRAND_RC = 2, IFA_STRAND_BOTH = 3 };

typedef struct {
    uint32_t abi_version;   /* must equal IFA_ABI_VERSION */
    int32_t device;         /* HIP device ordinal */
    uint64_t chunk_bases;   /* bases per device chunk; multiple of 32 in
                               [4096, 2^31]; fixes the device footprint */
    uint64_t hit_capacity;  /* hit records per device hit buffer (there are
                               two); 0 = auto: 1/32 of the device memory free
                               at ifa_create (hipMemGetInfo) over the two,
                               within [2^20, 2^26] records each. A full buffer
                               never loses hits: the chunk is re-scanned in
                               halves, and a buffer grows only if the 32
                               windows of one plane word x every query strand
                               alone overflow it */
    uint32_t strands;       /* IFA_STRAND_* */
    uint32_t n_policy;      /* IFA_N_SEPARATE | IFA_N_AS_MISMATCH */
    uint32_t sink;          /* IFA_SINK_RECORDS | IFA_SINK_COUNT_DIGEST */
    uint32_t host_threads;  /* packing threads; 0 = hardware concurrency */
    uint32_t work_capacity; /* filter work items per list (one item per wave
                               and batch of 32 query strands with a candidate
                               window); 0 = auto (2^22, or more when the
                               loaded queries are expected to need it on
                               random bases). A full list never loses work:
                               it grows and the filtered part of the pass
                               runs again */
    uint32_t flags;         /* IFA_FLAG_* bits; others must be 0 */
} ifa_config;

/* ifa_config.flags: replay scan passes from captured HIP graphs, one per
 * device chunk (resident chunk or stream slot), hit buffer and query-table
 * set. A pass is captured the second time its launch structure (kernels,
 * block sizes, LDS) repeats; later passes with other arguments (another
 * streamed chunk, another query set) update the graph's kernel nodes before
 * the replay. Results are identical. Set by ifa_config_default. */
#define IFA_FLAG_GRAPHS 1u
/* ifa_config.flags: also report the windows that overhang a contig end (see
 * the definition at the top). Off by default. */
#define IFA_FLAG_OVERHANG 2u
/* ifa_config.flags: indexed mode (Methods, "Algorithm Design"): a window is
 * reported only if it is a hit as defined at the top AND at least T of the
 * query strand's seeds occur error-free at the same offset of the window.
 * Seeds are the strand's k-mers at offsets 0, step, 2 step, ... with no N at
 * an unmasked position (a centre of `mask` bases of every k-mer is ignored);
 * a seed occurs error-free when the window's bases equal it at every
 * unmasked position. k is the longest candidate length whose MinHits is at
 * least 1 (else the shortest; a query shorter than every candidate uses
 * k = L); T = max(1, MinHits) for the strand's own seed count. MinHits is
 * the largest t such that, over `iters` Monte Carlo trials placing
 * min(maxSubs, span) substitutions uniformly at distinct positions of a
 * query modelled as V seeds spanning (V - 1) step + k bases, at least
 * prob_ppm / 10^6 of the trials leave t or more seeds error-free; at
 * prob_ppm = 10^6 it is the deterministic bound V - kEffective x maxSubs,
 * kEffective the most seeds one substitution can touch. Trials draw from
 * SplitMix64 (stream `seed`, draw n = mix64(seed + (n + 1) x golden gamma),
 * uniform positions by multiply-shift) through a partial Fisher-Yates
 * shuffle of a position array kept across trials. Not combined with
 * IFA_FLAG_OVERHANG. */
#define IFA_FLAG_INDEXED 4u
/* ifa_config.flags: choose the mode per query set (Discussion: the mode is
 * selected explicitly or automatically from the query count): a set of at
 * least ifa_index_params.auto_queries queries runs in indexed mode, a smaller
 * one by brute force. Not combined with IFA_FLAG_OVERHANG; IFA_FLAG_INDEXED
 * takes precedence. */
#define IFA_FLAG_AUTO_MODE 8u

/* One reported window (16 bytes). strand: 0 = +, 1 = - (reverse complement). */
typedef struct {
    uint32_t query;         /* index of the query in the last ifa_load_queries */
    uint32_t contig;        /* global contig ordinal, in stream order from 0 */
    int32_t pos;            /* 0-based leftmost forward coordinate in the contig
                               (negative: the window starts before the contig) */
    uint8_t strand;
    uint8_t n_ref;          /* reference non-ACGT bases in the window */
    uint16_t mismatches;    /* m as defined above */
} ifa_hit;

/* Counters since ifa_create (or the last ifa_reset_stats). */
typedef struct {
    uint64_t bases;          /* reference bases submitted for scanning */
    uint64_t chunks;         /* chunk scans submitted */
    uint64_t kernel_launches;/* scan passes (filter, resolve and dense kernels of one
                                chunk or word range), overflow re-scans included */
    uint64_t rescans;        /* re-scans caused by a full hit buffer */
    uint64_t hits;           /* hits found */
    double kernel_ms;        /* summed scan-pass time, HIP events on the compute
                                stream around the kernels of each pass */
    double h2d_ms;           /* summed host-to-device copy time of chunks */
    double pack_ms;          /* host wall time spent packing contigs */
    double filter_ms;        /* summed time of the filter kernel alone (the hot
                                loop) over the timed passes (timed_filter_passes),
                                HIP events on the compute stream; in a pass that
                                also has dense strands, the dense kernels run
                                beside it on a second stream, so this time and
                                dense_ms overlap */
    uint64_t filter_launches;/* filter kernel launches */
    uint64_t filter_windows; /* window starts the filter kernel evaluated (those of
                                waves holding a reference N are passed whole to the
                                resolve kernel and not counted) */
    uint64_t work_items;     /* work-list items the filter emitted */
    uint64_t graph_launches; /* scan passes replayed from a captured graph */
    uint64_t graph_updates;  /* of those, replays whose kernel arguments were updated
                                first (another streamed chunk or query set) */
    double edge_ms;          /* summed time of the overhanging-window kernel
                                (IFA_FLAG_OVERHANG) over the timed passes, HIP events */
    double dense_ms;         /* summed time of the dense-strand kernels (or, in
                                indexed mode, the seed kernel) over the timed passes,
                                HIP events */
    uint64_t filter_strand_windows;      /* sum over filter launches of the window
                                            starts evaluated x the filtered strands */
    uint64_t filter_half_strand_windows; /* of those, for strands in three-class tiles
                                            that run the first K step alone (maxSubs 0
                                            and similar: their windows tested on their
                                            first 16 - shift bases) */
    uint64_t timed_passes;   /* passes whose kernels were timed one by one: those
                                launched eagerly (a pass replayed from a captured graph
                                is timed as a whole, in kernel_ms, by events around the
                                graph launch; events recorded inside a graph misreport
                                the time of the kernels between them) */
    uint64_t timed_filter_passes; /* of those, passes with a filter launch */
} ifa_stats;

/* Fill *cfg with the defaults: device 0, 2^30-base chunks, automatic hit
 * capacity, both strands, IFA_N_SEPARATE, records sink, all host threads,
 * flags IFA_FLAG_GRAPHS. */
void ifa_config_default(ifa_config *cfg);

/* Create a context on cfg->device (cfg NULL = defaults). Allocates the fixed
 * device footprint: two chunk buffers of 0.5 byte per base plus hit buffers.
 * Errors: IFA_E_INVALID (bad config), IFA_E_DEVICE, IFA_E_NOMEM. */
ifa_status ifa_create(const ifa_config *cfg, ifa_ctx **out);

/* Load the query set, once before scanning (Methods, "Memory Management": the
 * query set is loaded once). n queries; seq[i] points to len[i] bytes;
 * max_subs[i] >= 0 (values above len[i] act as len[i]); max_n NULL means
 * floor(len[i] / 4) for every query (the 25% soft-clip default of Methods,
 * "Algorithm Design"), else max_n[i] >= 0.
 * Errors: IFA_E_TOO_LONG (len 0 or > IFA_MAX_QUERY_LEN), IFA_E_INVALID
 * (negative threshold, NULL pointer), IFA_E_STATE (chunks or hits still
 * pending: call ifa_collect_hits first). Resets count+digest statistics. */
ifa_status ifa_load_queries(ifa_ctx *ctx, uint32_t n, const uint8_t *const *seq,
                            const uint32_t *len, const int32_t *max_subs,
                            const int32_t *max_n);

/* Stream n_contigs contigs (seq[i] -> len[i] bytes, len[i] < 2^31) into the
 * scan. Contigs take global ordinals in call order; *first_ordinal (may be
 * NULL) receives the first one. Empty or short contigs take an ordinal and
 * yield no windows. Contigs are packed to 2-bit planes on host threads and
 * scanned asynchronously as device chunks fill; a contig longer than the room
 * left in a chunk continues in the next chunk, which repeats its last
 * IFA_MAX_QUERY_LEN - 1 bases so that every window is tested exactly once.
 * Errors: IFA_E_STATE (no queries loaded), IFA_E_INVALID, IFA_E_DEVICE. */
ifa_status ifa_scan_chunk(ifa_ctx *ctx, uint32_t n_contigs, const uint8_t *const *seq,
                          const uint64_t *len, uint32_t *first_ordinal);

/* A chunk of whole contigs packed by the caller (a producer that already
 * holds 2-bit data: the reference streams in on the fly, Methods, "Algorithm
 * Design" and "Memory Management"). Contigs lie back to back from base 0;
 * base x is bit x & 31 of word x >> 5 of the two code planes, with
 * A = (hi 0, lo 0), C = (0, 1), G = (1, 1), T = (1, 0) (bits 2 and 1 of the
 * base's ASCII letter, either case). Non-ACGT bases are given as N runs;
 * their plane bits are ignored, as are bits past n_bases in the last word. */
typedef struct {
    uint64_t n_bases;             /* <= ifa_config.chunk_bases */
    const uint32_t *hi, *lo;      /* ceil(n_bases / 32) words each */
    uint32_t n_contigs;
    uint32_t n_runs;
    const uint64_t *contig_len;   /* n_contigs lengths (< 2^31) adding up to n_bases;
                                     a contig of length 0 takes an ordinal only */
    const uint64_t *run_start;    /* n_runs N runs: chunk offsets, ascending */
    const uint32_t *run_len;      /* their lengths (>= 1); runs are disjoint and
                                     inside the chunk */
} ifa_packed_chunk;

/* Scan one caller-packed chunk: the same hits (and ordinals) as
 * ifa_scan_chunk of the same contigs as bytes, with every N-run base as 'N'.
 * Contigs take global ordinals in order (*first_ordinal, may be NULL, gets
 * the first); anything streamed by ifa_scan_chunk before is submitted first.
 * The planes are copied to the library's pinned staging before the call
 * returns; only the 2-bit planes and a list of the words holding an N or a
 * contig end cross to the device, whose N and contig-end planes are rebuilt
 * there. Errors: IFA_E_STATE (no queries loaded), IFA_E_INVALID (sizes, NULL
 * pointers, runs out of order or outside the chunk, lengths that do not add
 * up), IFA_E_DEVICE. */
ifa_status ifa_scan_packed(ifa_ctx *ctx, const ifa_packed_chunk *chunk, uint32_t *first_ordinal);

/* Wait for every submitted scan and hand out the hits found so far in
 * reference order: (contig, pos, strand, query) ascending, pos signed (Results, "Accuracy
 * Validation": output follows the reference stream). Writes at most cap
 * records to out; *n_written gets the count written and *n_remaining (may be
 * NULL) the count still held; call again to drain the rest. With the
 * count+digest sink no records exist and both counts are 0. */
ifa_status ifa_collect_hits(ifa_ctx *ctx, ifa_hit *out, uint64_t cap, uint64_t *n_written,
                            uint64_t *n_remaining);

/* Release everything the context owns. NULL-safe. */
void ifa_destroy(ifa_ctx *ctx);

/* Message of the last failed call on ctx ("" if none). The string belongs to
 * the context and lives until its next call. */
const char *ifa_last_error(const ifa_ctx *ctx);

/* Count+digest sink: waits for every submitted scan, then writes for each
 * loaded query the number of hits and the wrapping 64-bit sum over its hits of
 *   mix64(((contig << 32) | (uint32_t)pos) ^ (aux << 45)),
 *   aux = strand | (mismatches << 1) | (n_ref << 10),
 * mix64 being the SplitMix64 output finaliser (shifts 30, 27, 31; multipliers
 * 0xBF58476D1CE4E5B9, 0x94D049BB133111EB). count and digest are arrays of the
 * loaded query count. Errors: IFA_E_STATE (records sink or no queries). */
ifa_status ifa_query_stats(ifa_ctx *ctx, uint64_t *count, uint64_t *digest);

/* Device-resident reference: pack contigs into device chunks that stay in
 * device memory (one chunk buffer per chunk_bases of reference) so that
 * later query sets can be scanned without copying the reference again.
 * Ordinals come from the same counter as ifa_scan_chunk. Errors: IFA_E_NOMEM
 * when device memory runs out (what was loaded before the call stays). */
ifa_status ifa_ref_load(ifa_ctx *ctx, uint32_t n_contigs, const uint8_t *const *seq,
                        const uint64_t *len, uint32_t *first_ordinal);

/* Scan every resident chunk with the loaded queries; hits are collected as
 * for ifa_scan_chunk. Errors: IFA_E_STATE (no queries or no resident chunk). */
ifa_status ifa_scan_resident(ifa_ctx *ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the scan of
 * ifa_scan_resident with nothing allocated. The pass counters and the filter
 * work list live in a fixed static device array of the library (16 MiB + 256
 * bytes per device, held until the process ends) instead of context memory,
 * and the hit records go straight to the caller's device buffer d_hits of cap
 * records (records sink; in no particular order, each window once, the same
 * set ifa_collect_hits would hand out after ifa_scan_resident). *n_hits gets
 * the number of hits found. Synchronous: returns when the scan is done; no
 * hits are left pending in the context. With the count+digest sink the hits
 * go to the per-query counters as usual (read them with ifa_query_stats);
 * d_hits may then be NULL and *n_hits is 0.
 * The static array is shared by every context on the device and keeps the
 * last call's contents (the call clears what it needs first): calls that
 * overlap in time on one device race and must not be made.
 * Errors: IFA_E_NOMEM when more than cap records were found (*n_hits gets the
 * count needed; d_hits then holds cap of them); IFA_E_INVALID (NULL n_hits or
 * d_hits, or more than 8 * 2^20 filtered query strands, which the static work
 * list cannot hold); IFA_E_STATE (no queries, no resident reference, scans or
 * hits pending, or the variant was changed after the queries were loaded so
 * its matrix-filter operands would have to be built). */
ifa_status ifa_scan_resident_into(ifa_ctx *ctx, ifa_hit *d_hits, uint64_t cap, uint64_t *n_hits);

/* Free the resident reference. Errors: IFA_E_STATE while scans are pending. */
ifa_status ifa_ref_release(ifa_ctx *ctx);

/* Resident reference size: bases (*bases) in *chunks device chunks. */
ifa_status ifa_ref_info(const ifa_ctx *ctx, uint64_t *bases, uint32_t *chunks);

/* Counters (see ifa_stats). ifa_get_stats waits for submitted work first. */
ifa_status ifa_get_stats(ifa_ctx *ctx, ifa_stats *out);

/* Turn the capture and replay of scan passes as HIP graphs (IFA_FLAG_GRAPHS)
 * on (enable != 0) or off for the context's later scans; graphs captured so
 * far are kept. With it off every pass is launched eagerly and its kernels
 * are timed one by one in the statistics. Waits for submitted work first.
 * Errors: IFA_E_INVALID (ctx NULL). */
ifa_status ifa_set_graphs(ifa_ctx *ctx, int enable);

/* Run the dense-strand kernels of a pass that also has filtered strands on a
 * second stream beside the filter and resolve kernels (enable != 0, the
 * default), or after them on one stream. Results are identical; beside each
 * other the kernels share the device, so each one's time in the statistics
 * covers the other's work too, and with it off each kernel is timed alone.
 * Passes captured in the other arrangement are captured again. Waits for
 * submitted work first. Errors: IFA_E_INVALID (ctx NULL). */
ifa_status ifa_set_overlap(ifa_ctx *ctx, int enable);
ifa_status ifa_reset_stats(ifa_ctx *ctx);

/* Query strands of the loaded set (*n_strands) and how many of them take the
 * filter kernel (*n_filtered); the rest are predicted hit-dense and are
 * resolved directly. */
ifa_status ifa_query_partition(const ifa_ctx *ctx, uint32_t *n_strands, uint32_t *n_filtered);

/* Device memory held by the context, in bytes: stream chunk buffers, hit
 * buffers, work lists, query tables, counters and any resident reference. */
ifa_status ifa_device_footprint(const ifa_ctx *ctx, uint64_t *bytes);

/* Indexed-mode parameters (IFA_FLAG_INDEXED, IFA_FLAG_AUTO_MODE), with the paper's defaults
 * (Methods, "Algorithm Design"): candidate seed lengths 8, 9, 10, 12, 14;
 * no mask; step 1; probability 99.9 %; 200,000 trials; a fixed seed. */
#define IFA_MAX_SEED_KS 8
typedef struct {
    uint32_t n_k;                   /* candidate lengths in k[], 1..IFA_MAX_SEED_KS */
    uint32_t k[IFA_MAX_SEED_KS];    /* each in [mask + 1, 16] */
    uint32_t mask;                  /* masked centre of every k-mer, bases */
    uint32_t step;                  /* seed sampling step, >= 1 */
    uint32_t prob_ppm;              /* MinHits probability x 10^6, <= 10^6 */
    uint32_t auto_queries;          /* IFA_FLAG_AUTO_MODE: indexed from this many
                                       queries on (default: the measured crossover) */
    uint64_t iters;                 /* Monte Carlo trials, >= 1 */
    uint64_t seed;                  /* SplitMix64 stream of the trials */
} ifa_index_params;

void ifa_index_params_default(ifa_index_params *p);

/* Set the parameters used by the next ifa_load_queries of an indexed-mode or
 * auto-mode context. Errors: IFA_E_INVALID (bad values, or a context with
 * neither flag). */
ifa_status ifa_set_index_params(ifa_ctx *ctx, const ifa_index_params *p);

/* Seeds chosen for the loaded queries: k[j] per query and thr[2 j + s] per
 * query and strand (0 for a strand not scanned). Arrays of the loaded query
 * count (and twice that). Errors: IFA_E_STATE (no queries, or not indexed). */
ifa_status ifa_query_seeds(const ifa_ctx *ctx, uint32_t *k, uint32_t *thr);

/* Mode of the loaded query set: *indexed = 1 for indexed mode, 0 for brute
 * force. Errors: IFA_E_STATE (no queries loaded). */
ifa_status ifa_query_mode(const ifa_ctx *ctx, uint32_t *indexed);

/* Kernel variants: tile shapes of the scan kernel (windows per lane, query
 * strands per loop iteration, workgroup size) and the arithmetic of the
 * filter kernel (encoding 0: vector-ALU bit operations; 1: fp4 matrix cores
 * on four-class one-hot codes; 2: fp4 matrix cores on three-class codes; 3:
 * as 2, and the dense query strands of at most 32 bases are counted on the
 * matrix cores too, on waves without an N or a contig end).
 * Every variant computes the same hits; they differ only in speed. Any
 * output pointer may be NULL. A new context starts with a three-class
 * matrix-core variant; ifa_get_variant names it. */
uint32_t ifa_variant_count(void);
ifa_status ifa_variant_info(uint32_t v, uint32_t *windows_per_lane, uint32_t *queries_per_iter,
                            uint32_t *workgroup, uint32_t *encoding);
ifa_status ifa_set_variant(ifa_ctx *ctx, uint32_t v);
ifa_status ifa_get_variant(const ifa_ctx *ctx, uint32_t *v);

/* Autotuner: time every variant on a calibration chunk of calib_bases
 * uniform random bases (0 = 64 Mi) with the loaded queries, median of reps
 * launches (0 = 3), and select the fastest for this context. Each pass is
 * timed as a scan runs it (dense kernels beside the filter while
 * ifa_set_overlap is on). cache_path (may be NULL): a text file of
 * "key variant ms" lines keyed by device architecture, query-strand count
 * band, longest query in words, threshold band and the overlap setting; a
 * cached key is used without timing, a new result is appended.
 * *chosen (may be NULL) gets the variant; ms_per_variant (may be NULL) gets
 * ifa_variant_count() medians (-1 when taken from the cache). Hits found on
 * the calibration chunk are discarded. Errors: IFA_E_STATE (no queries, or
 * scans pending). */
ifa_status ifa_autotune(ifa_ctx *ctx, uint64_t calib_bases, uint32_t reps, const char *cache_path,
                        uint32_t *chosen, double *ms_per_variant);

/* ------------------------------------------------------------------------
 * Serving loop: continuous batching over a device-resident reference.
 *
 * Query sets ("requests") arrive at any time through ifa_server_submit. Each
 * ifa_server_step scans one resident chunk, the one under a rotating cursor,
 * with the query strands of every admitted request together, so the work of
 * concurrent requests shares the same kernel launches. A request admitted at
 * a step completes after one full revolution over the resident chunks; its
 * hits are exactly those of a plain scan of that query set alone (same
 * records, same reference order). Steps are pipelined: a step submits its
 * chunk's scan, then waits for the previous step's scan and routes its hits
 * (a step that submits nothing drains the last one), so a request completes
 * within the step that submits its last chunk.
 *
 * Admission keeps the admitted query count under max_active_queries and the
 * hits one step can produce under hit_budget records: a request reserves, per
 * chunk, its expected hits on iid uniform bases (each base matches with
 * probability 1/4: sum over strands of chunk bases x P(Bin(L, 3/4) <= k))
 * plus six standard deviations and 1,024 records. The context's hit buffers
 * grow to the admitted reservation; a request alone is always admitted (a
 * chunk whose hits overflow is re-scanned in halves, as for any scan). A
 * server borrows its context: the context must hold a resident reference
 * (ifa_ref_load), use the records sink, and must not be used for other scans
 * while the server exists.
 * ------------------------------------------------------------------------ */
typedef struct ifa_server ifa_server;

typedef struct {
    uint32_t max_active_queries;  /* default 4096 */
    uint32_t reserved;            /* must be 0 */
    uint64_t hit_budget;          /* records per step; 0 (default) = a quarter of the
                                     device memory free at ifa_server_create
                                     (hipMemGetInfo), over two 16-byte record buffers */
} ifa_server_config;

typedef struct {
    uint32_t pending;         /* submitted, not yet admitted */
    uint32_t active;          /* admitted, chunks left to scan */
    uint32_t active_queries;
    uint32_t done_waiting;    /* completed, hits not yet taken */
    uint64_t steps;
    uint64_t completed;
    double step_ms;           /* host wall time inside steps */
    uint32_t cursor;          /* next resident chunk */
    uint32_t chunks;          /* resident chunks */
    uint64_t hit_budget;      /* records per step in force */
    uint64_t hits_reserved;   /* records reserved by the admitted requests */
    uint32_t in_flight;       /* submitted scans whose hits are not routed yet */
    uint32_t finishing;       /* requests with every chunk submitted, hits not all routed */
} ifa_server_stats;

void ifa_server_config_default(ifa_server_config *cfg);
ifa_status ifa_server_create(ifa_ctx *ctx, const ifa_server_config *cfg, ifa_server **out);
void ifa_server_destroy(ifa_server *srv);   /* NULL-safe; pending requests are dropped */

/* Queue a request of n queries (same arguments as ifa_load_queries). Hits
 * report query indices within the request. *request_id (may be NULL) gets
 * its id (ids count up from 1). */
ifa_status ifa_server_submit(ifa_server *srv, uint32_t n, const uint8_t *const *seq,
                             const uint32_t *len, const int32_t *max_subs, const int32_t *max_n,
                             uint64_t *request_id);

/* Admit what fits, submit the scan of the chunk under the cursor for every
 * admitted request and advance the cursor; then wait for the previous step's
 * scan and route its hits (with no request admitted, only the latter). Does
 * nothing when nothing is admitted or in flight. */
ifa_status ifa_server_step(ifa_server *srv, uint32_t *n_active, uint32_t *n_done_waiting);

/* The oldest completed request not yet taken: *request_id (0 if none) and
 * its hit count. */
ifa_status ifa_server_poll(ifa_server *srv, uint64_t *request_id, uint64_t *n_hits);

/* Copy the hits of the request ifa_server_poll returned (cap >= its hit
 * count) in reference order, and release it. */
ifa_status ifa_server_take(ifa_server *srv, uint64_t request_id, ifa_hit *out, uint64_t cap);

ifa_status ifa_server_info(const ifa_server *srv, ifa_server_stats *out);

/* ------------------------------------------------------------------------
 * SAM text. The aligner streams the reference, so its SAM output is
 * headerless and a separate header is concatenated in front of it (Methods,
 * "Output Format"). A query's primary alignment is its first valid alignment
 * in reference order, every other one is secondary (Results, "Accuracy
 * Validation"); queries without a hit get no line. Host code only.
 *
 * One line per hit: QNAME, FLAG (16 = reverse-complement strand, 256 =
 * secondary), RNAME, POS (1-based first aligned base), MAPQ 255, CIGAR
 * [aS]mM[bS] (a, b = bases off the contig's left / right end, IFA_FLAG_OVERHANG),
 * RNEXT *, PNEXT 0, TLEN 0, SEQ (the strand sequence as compared: the query or
 * its reverse complement, upper case, N for non-ACGT), QUAL *, NM:i
 * (mismatches over the aligned bases) and XN:i (reference Ns over the aligned
 * bases). The header holds @HD VN:1.6 SO:coordinate, one @SQ per contig in
 * ordinal order and @PG ID:ifa.
 * ------------------------------------------------------------------------ */
typedef struct ifa_sam ifa_sam;

/* A writer for the hits of one query set: seq/len as given to
 * ifa_load_queries, names[j] the query names (non-empty, no tab or newline),
 * n_policy the context's IFA_N_* policy. Copies what it needs.
 * Errors: IFA_E_INVALID, IFA_E_NOMEM. */
ifa_status ifa_sam_create(uint32_t n_queries, const uint8_t *const *seq, const uint32_t *len,
                          const char *const *names, uint32_t n_policy, ifa_sam **out);

/* NULL-safe. */
void ifa_sam_destroy(ifa_sam *w);

/* Message of the writer's last failed call ("" if none); lives until its next call. */
const char *ifa_sam_last_error(const ifa_sam *w);

/* Name and length of contigs first_ordinal .. first_ordinal + n - 1, the
 * ordinals ifa_scan_chunk / ifa_ref_load gave them; added in ordinal order
 * without gaps. Errors: IFA_E_INVALID (order, name, len >= 2^31). */
ifa_status ifa_sam_add_contigs(ifa_sam *w, uint32_t first_ordinal, uint32_t n,
                               const char *const *names, const uint64_t *len);

/* The header for the contigs added so far. *n_bytes receives its size; with
 * buf == NULL nothing else happens, else it is copied to buf (no NUL) and
 * IFA_E_INVALID is returned when cap is smaller. */
ifa_status ifa_sam_header(const ifa_sam *w, char *buf, uint64_t cap, uint64_t *n_bytes);

/* Format hits (in reference order, as ifa_collect_hits hands them out; the
 * order continues across calls) into buf as whole lines, no NUL. Stops at the
 * first line that does not fit or at the first invalid hit; *n_consumed and
 * *n_bytes tell how far it got. The primary/secondary state advances only
 * over consumed hits. Errors (nothing consumed): IFA_E_INVALID when the first
 * hit is invalid (query or contig unknown, out of reference order, window not
 * on its contig) or its line alone exceeds cap. */
ifa_status ifa_sam_format(ifa_sam *w, const ifa_hit *hits, uint64_t n, char *buf, uint64_t cap,
                          uint64_t *n_consumed, uint64_t *n_bytes);

#ifdef __cplusplus
}
#endif

#endif /* IFA_H */
