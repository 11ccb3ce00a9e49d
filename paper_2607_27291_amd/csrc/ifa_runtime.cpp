// ifa_runtime.cpp -- host runtime of libifa.so (the C ABI in include/ifa.h).
//
// Streaming architecture (Methods, "Algorithm Design" and "Memory
// Management"): contigs arrive on the fly; the host packs them into 2-bit
// planes in pinned staging buffers; full chunks are copied to one of two
// device chunk buffers and scanned while the host packs the next one. Device
// memory is fixed at creation (two chunk buffers, two hit buffers), so it does
// not depend on the total reference size nor on the largest contig: a contig
// that does not fit is split, and the next chunk repeats its last kCarry bases.
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ifa.h"
#include "ifa_dev.h"
#include "ifa_seed.h"

namespace ifa {
// (rec != nullptr: the launches are recorded in rec instead of issued)
hipError_t launch_filter(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec = nullptr);
hipError_t launch_resolve(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec = nullptr);
hipError_t launch_dense(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec = nullptr);
hipError_t launch_edge(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec = nullptr);
hipError_t launch_seed(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec = nullptr);
hipError_t launch_clear_u64(unsigned long long *p, uint32_t n, hipStream_t s);
hipError_t launch_expand(uint32_t *planes, uint64_t stride, uint8_t *nflag, uint32_t used,
                         uint32_t total, const uint4 *list, uint32_t n_list, hipStream_t s);
hipError_t launch_clear_u32(unsigned int *p, uint32_t n, hipStream_t s);
hipError_t launch_seed_bitmap(const uint2 *ent, uint32_t n, uint32_t *bm, uint32_t words,
                              uint32_t key_bits, hipStream_t s);
void *scratch_address(int device, hipError_t *err);
uint32_t variant_count();
uint32_t variant_default();
void variant_shape(uint32_t v, uint32_t *windows, uint32_t *qunroll, uint32_t *wg, uint32_t *enc);
}  // namespace ifa

using namespace ifa;

namespace {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

struct Failure {
    ifa_status st;
    std::string msg;
};

[[noreturn]] void fail(ifa_status st, const std::string &msg) { throw Failure{st, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
            fail(IFA_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
        fail(IFA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// byte -> base code, anything other than A/C/G/T/a/c/g/t is 4 (N). The 2-bit
// code (hi, lo) of a base is bits 2 and 1 of its ASCII byte: A=00, C=01,
// G=11, T=10, in either case; complementing a base flips hi.
struct CodeTable {
    uint8_t c[256];
    CodeTable()
    {
        std::memset(c, 4, sizeof c);
        for (const char *p = "ACGTacgt"; *p; p++) c[(uint8_t)*p] = ((uint8_t)*p >> 1) & 3u;
    }
};
const CodeTable kCode;

void parallel_for(unsigned threads, size_t n, const std::function<void(size_t)> &fn)
{
    if (n == 0) return;
    unsigned t = std::max(1u, std::min<unsigned>(threads, (unsigned)n));
    if (t == 1) {
        for (size_t i = 0; i < n; i++) fn(i);
        return;
    }
    std::atomic<size_t> next{0};
    auto body = [&]() {
        for (;;) {
            size_t i = next.fetch_add(1);
            if (i >= n) break;
            fn(i);
        }
    };
    std::vector<std::thread> th;
    th.reserve(t - 1);
    for (unsigned i = 1; i < t; i++) th.emplace_back(body);
    body();
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// pinned / device buffers
// ---------------------------------------------------------------------------

template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count, const char *what)
    {
        release();
        if (count == 0) count = 1;
        hip_check(hipMalloc((void **)&p, count * sizeof(T)), what);
        n = count;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

template <class T>
struct HostBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count, const char *what)
    {
        release();
        if (count == 0) count = 1;
        hip_check(hipHostMalloc((void **)&p, count * sizeof(T), hipHostMallocDefault), what);
        n = count;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    ~HostBuf() { release(); }
};

// ---------------------------------------------------------------------------
// host staging chunk
// ---------------------------------------------------------------------------

// A pending copy of contig bytes into the staging planes.
struct PackTask {
    const uint8_t *src;
    uint64_t dst;     // chunk-local base offset
    uint64_t n;
};

struct Staging {
    HostBuf<uint32_t> planes;       // hi, lo and nm planes of plane_words each
    HostBuf<uint4> list;            // sparse N / piece-end words (seal)
    uint32_t n_list = 0;
    std::vector<Piece> pieces;
    std::vector<PackTask> tasks;    // not yet packed
    uint64_t len = 0;               // bases used
    uint32_t own_from = 0;
    uint64_t packed_to = 0;         // bases [0, packed_to) are packed
    hipEvent_t copied = nullptr;    // H2D from this staging finished
    bool copy_pending = false;
};

// Device chunk: planes + piece table, either a stream slot or resident.
// A captured scan pass of one resident chunk into one hit buffer: replayed
// while the pass's launch arguments stay the same (the query tables' content
// may change; their addresses and sizes may not).
// A captured scan pass of one device chunk into one hit buffer with one
// set of query tables. The pass is captured the second time its launch
// structure (kernels, block sizes, LDS) repeats and replayed after that; when
// only arguments or grid sizes differ (another streamed chunk, other query
// counts) its kernel nodes are updated in place before the replay.
struct PassGraph {
    ScanArgs args{};              // arguments the graph holds (or the last eager pass had)
    std::vector<ScanLaunch> plan; // the scan-kernel launches of that pass
    bool seen = false;            // plan holds a pass that ran
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> knodes;   // the scan-kernel nodes, in plan order
    bool forked = false;          // dense kernels on the second stream
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        knodes.clear();
        plan.clear();
        seen = false;
        forked = false;
    }
};

struct DevChunk {
    DevBuf<uint32_t> planes;      // 4 planes of `stride` words each
    DevBuf<uint8_t> nflag;        // N flag per 32-word block (nflag_blocks(stride))
    DevBuf<uint4> sparse;         // the uploaded sparse N / piece-end list
    DevBuf<Piece> pieces;
    uint64_t stride = 0;
    uint64_t len = 0;
    uint32_t own_from = 0;
    uint32_t n_pieces = 0;
    hipEvent_t free_ev = nullptr;   // last kernel reading it finished
    bool resident = false;
    PassGraph graph[2][2];          // per hit buffer and query-table set (resident chunks)
    ~DevChunk()
    {
        for (auto &g : graph)
            for (auto &x : g) x.reset();
    }
};

// A submitted scan of one device chunk whose hits are not yet retired.
struct Job {
    DevChunk *chunk = nullptr;
    int hitbuf = 0;
    ScanArgs args{};                      // the pass's launch arguments (re-scans reuse
                                          // them: the query tables they point to stay
                                          // valid until the job is retired)
    hipEvent_t k0 = nullptr, kf = nullptr, k1 = nullptr;  // start / filter end / stop
    hipEvent_t kd = nullptr, kx = nullptr;                // dense kernels start / end
    hipEvent_t ke = nullptr;                              // overhang kernel start
    hipEvent_t done = nullptr;              // hit count copied to the host
    uint32_t n_half = 0;                    // filtered strands in half-step tiles
    bool split_timed = false;               // kf, kd, kx, ke recorded (eager launches)
    bool active = false;
};

}  // namespace

struct ifa_ctx {
    ifa_config cfg{};
    std::string err;
    unsigned threads = 1;
    uint64_t plane_words = 0;

    hipStream_t copy_s = nullptr, comp_s = nullptr;
    // the dense kernels of a pass that also has filtered strands run on
    // dense_s, beside the filter and resolve kernels (fork and join events)
    hipStream_t dense_s = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    bool overlap = true;   // ifa_set_overlap

    // kernel variant (autotuner or caller's choice)
    uint32_t variant = variant_default();
    std::vector<double> tune_ms;

    // queries
    bool have_queries = false;
    uint32_t n_queries = 0;
    uint32_t lmax = 0;
    std::vector<QSDesc> h_qs;         // sparse strands first, then dense
    uint32_t n_sparse = 0;
    std::vector<uint32_t> h_qwords;
    // device query tables, uploaded together through a pinned staging arena:
    // strand descriptors, packed words and the three-class filter's words per
    // column tile
    // Two sets of tables alternate between query sets (tab), so that a new
    // set can be uploaded while passes of the previous one are still queued;
    // `staged` marks the end of the last copy out of each pinned staging.
    int tab = 0;
    DevBuf<uint8_t> d_qarena[2];
    HostBuf<uint8_t> h_qarena[2];
    hipEvent_t qstaged[2] = {nullptr, nullptr};
    const QSDesc *dq_qs = nullptr;
    const uint32_t *dq_words = nullptr;
    const uint32_t *dq_mq3w = nullptr;
    // the matrix-core filters' B operands and required match counts, one
    // arena per form (index 0: four-class, 1: three-class), built when a
    // pass first needs that form for the loaded query set
    std::vector<uint8_t> h_fw;        // filter words of each strand (device order)
    bool mq_ready[2] = {false, false};
    DevBuf<uint8_t> d_mqarena[2][2];      // [tab][form]
    HostBuf<uint8_t> h_mqarena[2][2];
    hipEvent_t mqstaged[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    const uint4 *dq_mqb = nullptr, *dq_mq3b = nullptr;
    const float *dq_mqt = nullptr, *dq_mq3t = nullptr;
    // dense strands counted on the matrix cores on clean waves (three-class
    // variants): [n_dm0, n_qs), all of at most 32 bases, and their operands
    uint32_t n_dm0 = 0;
    bool dm_ready = false;
    const uint4 *dq_dmb = nullptr;
    const float *dq_dmt = nullptr;
    uint32_t mq3_words = 1;           // most prefix words of any three-class column tile
    uint32_t mq3_two_batches = 0;     // leading batches holding a two-word tile
    uint32_t n_half_strands = 0;      // sparse strands in half-step three-class tiles
    uint32_t edge_pmin = 0;           // overhang kernel: pieces per wave (ScanArgs.edge_pmin)
    DevBuf<unsigned long long> d_qcount, d_qdigest;
    // indexed mode: parameters, MinHits cache, the query set's seeds and
    // their device tables
    SeedParams seedp;
    bool indexed = false;             // mode of the loaded query set
    MinHitsCache mh_cache;
    SeedBuild seeds;
    DevBuf<SeedInfo> d_seed_info;
    DevBuf<uint32_t> d_seed_dir[kMaxSeedCfg], d_seed_ent[kMaxSeedCfg], d_seed_bm[kMaxSeedCfg];
    DevBuf<SeedTable> d_seed_tab;     // [kMaxSeedCfg]

    // streaming
    Staging stage[2];
    int cur = 0;                      // staging being filled
    DevChunk slot[2];
    uint64_t chunk_seq = 0;           // chunks submitted to stream slots
    uint32_t next_ordinal = 0;

    // hits
    DevBuf<uint4> d_hits[2];
    // pass counters, 16 bytes per hit buffer hb: [2 hb] hit count, [2 hb + 1]
    // work items (low word) and waves handed to the resolve kernel (high)
    DevBuf<unsigned long long> d_ctr;   // [4]
    HostBuf<unsigned long long> h_ctr;  // [4], pinned
    uint64_t hit_cap = 0;             // configured records per hit buffer
    uint64_t buf_cap[2] = {0, 0};     // current records per hit buffer
    DevBuf<WorkItem> work[2];         // sparse-path work lists, one per hit buffer
    uint32_t work_cap[2] = {0, 0};
    uint32_t work_want = 0;           // capacity both work lists grow to before a launch
    Job jobs[2];
    uint64_t job_seq = 0;
    std::vector<ifa_hit> hits;        // retired, not yet handed out
    bool hits_sorted = true;
    uint64_t drain_pos = 0;

    // resident reference
    std::vector<std::unique_ptr<DevChunk>> resident;
    uint64_t resident_bases = 0;

    // device address of the static scratch array (allocation-free entry point)
    uint8_t *scratch = nullptr;

    // stats
    ifa_stats st{};
    hipEvent_t h2d0 = nullptr, h2d1 = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> h2d_pending;
};

namespace {

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------

uint32_t *plane(ifa_ctx *c, Staging &s, int k) { return s.planes.p + (size_t)k * c->plane_words; }

// One plane word from 32 bytes: hi = bit 2 of each byte, lo = bit 1, n = 1
// where the byte is not A/C/G/T/a/c/g/t.
__attribute__((target("avx2"))) void pack32_avx2(const uint8_t *p, uint32_t *h, uint32_t *l,
                                                 uint32_t *n)
{
    const __m256i v = _mm256_loadu_si256((const __m256i *)p);
    *h = (uint32_t)_mm256_movemask_epi8(_mm256_slli_epi16(v, 5));
    *l = (uint32_t)_mm256_movemask_epi8(_mm256_slli_epi16(v, 6));
    const __m256i f = _mm256_or_si256(v, _mm256_set1_epi8(0x20));   // fold case
    __m256i ok = _mm256_cmpeq_epi8(f, _mm256_set1_epi8('a'));
    ok = _mm256_or_si256(ok, _mm256_cmpeq_epi8(f, _mm256_set1_epi8('c')));
    ok = _mm256_or_si256(ok, _mm256_cmpeq_epi8(f, _mm256_set1_epi8('g')));
    ok = _mm256_or_si256(ok, _mm256_cmpeq_epi8(f, _mm256_set1_epi8('t')));
    *n = ~(uint32_t)_mm256_movemask_epi8(ok);
}

void pack32_scalar(const uint8_t *p, uint32_t cnt, uint32_t b0, uint32_t *h, uint32_t *l,
                   uint32_t *n)
{
    uint32_t hh = 0, ll = 0, nn = 0;
    for (uint32_t i = 0; i < cnt; i++) {
        const uint32_t b = p[i], bit = 1u << (b0 + i);
        if (kCode.c[b] == 4) nn |= bit;
        if (b & 4u) hh |= bit;
        if (b & 2u) ll |= bit;
    }
    *h = hh;
    *l = ll;
    *n = nn;
}

const bool kHaveAvx2 = __builtin_cpu_supports("avx2");

// Pack bases [dst, dst + n) of the chunk from src. Words are written whole,
// except the first word, whose bits below `dst` are kept when keep_low (they
// belong to bases packed earlier). hi/lo bits at N positions are whatever the
// byte holds: every reader masks N positions with the N plane.
void pack_range(ifa_ctx *c, Staging &s, uint64_t dst, const uint8_t *src, uint64_t n,
                bool keep_low)
{
    uint32_t *H = plane(c, s, 0), *Lo = plane(c, s, 1), *N = plane(c, s, 2);
    uint64_t x = dst, end = dst + n;
    while (x < end) {
        const uint64_t w = x >> 5;
        const uint32_t b0 = (uint32_t)(x & 31);
        const uint64_t wend = std::min<uint64_t>(end, (w + 1) << 5);
        const uint8_t *p = src + (x - dst);
        const uint32_t cnt = (uint32_t)(wend - x);
        uint32_t h, l, nn;
        if (cnt == 32 && kHaveAvx2)
            pack32_avx2(p, &h, &l, &nn);
        else
            pack32_scalar(p, cnt, b0, &h, &l, &nn);
        if (b0 != 0 && keep_low) {
            const uint32_t keep = (1u << b0) - 1u;
            H[w] = (H[w] & keep) | h;
            Lo[w] = (Lo[w] & keep) | l;
            N[w] = (N[w] & keep) | nn;
        } else {
            H[w] = h;
            Lo[w] = l;
            N[w] = nn;
        }
        x = wend;
    }
}

// Pack every pending task of staging s, in parallel over word-aligned spans.
void pack_pending(ifa_ctx *c, Staging &s)
{
    if (s.tasks.empty()) return;
    double t0 = now_ms();
    // Tasks are back to back in chunk order. The first word of the whole
    // region may hold bits packed by an earlier call; every later word is
    // written whole by exactly one worker.
    const uint64_t region0 = s.tasks.front().dst;
    const uint64_t region1 = s.tasks.back().dst + s.tasks.back().n;
    const uint64_t span = 1ull << 20;   // bases per work item (multiple of 32)
    const uint64_t a0 = region0 & ~31ull;
    const size_t items = (size_t)((region1 - a0 + span - 1) / span);
    std::vector<PackTask> &T = s.tasks;
    parallel_for(c->threads, items, [&](size_t it) {
        uint64_t lo = std::max(region0, a0 + (uint64_t)it * span);
        uint64_t hi = std::min(region1, a0 + (uint64_t)(it + 1) * span);
        if (lo >= hi) return;
        // first task overlapping [lo, hi)
        size_t k = (size_t)(std::upper_bound(T.begin(), T.end(), lo,
                                             [](uint64_t v, const PackTask &t) {
                                                 return v < t.dst;
                                             }) - T.begin());
        if (k > 0) k--;
        for (; k < T.size() && T[k].dst < hi; k++) {
            uint64_t s0 = std::max(lo, T[k].dst), s1 = std::min(hi, T[k].dst + T[k].n);
            if (s0 >= s1) continue;
            // keep earlier bits only in the very first word of the region;
            // bits of a word shared by two tasks are packed in task order by
            // this same worker
            bool keep = (s0 == region0) || (s0 != lo);
            pack_range(c, s, s0, T[k].src + (s0 - T[k].dst), s1 - s0, keep);
        }
    });
    s.packed_to = region1;
    s.tasks.clear();
    c->st.pack_ms += now_ms() - t0;
}

// Grow a pinned list to hold n entries (its contents are not kept).
void reserve_list(HostBuf<uint4> &l, size_t n)
{
    if (l.n < n) l.alloc(std::max<size_t>(n, l.n * 2), "pinned sparse list");
}

// The sparse list of a chunk: (word, nm, em, 0) for every used word that
// holds an N bit or a piece end, in word order. nword: the sorted words with
// an N bit and their nm values; ends: the sorted piece-end words and bits.
uint32_t merge_sparse(const std::vector<std::pair<uint32_t, uint32_t>> &nword,
                      const std::vector<std::pair<uint32_t, uint32_t>> &ends, HostBuf<uint4> &out)
{
    reserve_list(out, nword.size() + ends.size() + 1);
    size_t i = 0, j = 0, n = 0;
    while (i < nword.size() || j < ends.size()) {
        uint4 e{0u, 0u, 0u, 0u};
        if (j >= ends.size() || (i < nword.size() && nword[i].first < ends[j].first)) {
            e.x = nword[i].first;
            e.y = nword[i++].second;
        } else if (i >= nword.size() || ends[j].first < nword[i].first) {
            e.x = ends[j].first;
            e.z = ends[j++].second;
        } else {
            e.x = nword[i].first;
            e.y = nword[i++].second;
            e.z = ends[j++].second;
        }
        out.p[n++] = e;
    }
    return (uint32_t)n;
}

// Piece-end words of a chunk (pieces sorted by start), the chunk tail's bits
// past its last base included (they read as N and as piece ends).
std::vector<std::pair<uint32_t, uint32_t>> piece_end_words(const std::vector<Piece> &pieces,
                                                         uint64_t len)
{
    std::vector<std::pair<uint32_t, uint32_t>> ends;
    auto add = [&](uint32_t w, uint32_t bits) {
        if (!ends.empty() && ends.back().first == w) ends.back().second |= bits;
        else ends.emplace_back(w, bits);
    };
    for (const Piece &p : pieces) {
        const uint64_t last = p.start + p.len - 1;
        add((uint32_t)(last >> 5), 1u << (last & 31));
    }
    if (len & 31) add((uint32_t)(len >> 5), ~((1u << (len & 31)) - 1u));
    return ends;
}

// Finish the staging chunk: bits past the last base (hi = lo = 0, N) and the
// sparse list of N and piece-end words. The device rebuilds its nm and em
// planes and the padding from the list (upload).
void seal(ifa_ctx *c, Staging &s)
{
    uint32_t *H = plane(c, s, 0), *Lo = plane(c, s, 1), *N = plane(c, s, 2);
    const uint64_t used = (s.len + 31) >> 5;
    if (s.len & 31) {
        const uint64_t w = s.len >> 5;
        const uint32_t tail = ~((1u << (s.len & 31)) - 1u);
        H[w] &= ~tail;
        Lo[w] &= ~tail;
        N[w] |= tail;
    }
    // words with an N bit, found in parallel over spans of the N plane
    const uint64_t span = 1ull << 20;
    const size_t parts = (size_t)((used + span - 1) / span);
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> found(parts);
    parallel_for(c->threads, parts, [&](size_t i) {
        const uint64_t w1 = std::min<uint64_t>(used, (i + 1) * span);
        for (uint64_t w = i * span; w < w1; w++)
            if (N[w]) found[i].emplace_back((uint32_t)w, N[w]);
    });
    std::vector<std::pair<uint32_t, uint32_t>> nword;
    for (auto &f : found) nword.insert(nword.end(), f.begin(), f.end());
    s.n_list = merge_sparse(nword, piece_end_words(s.pieces, s.len), s.list);
}

uint64_t words_with_pad(uint64_t len) { return ((len + 31) >> 5) + kPadWords; }

// P(Bin(n, p) <= k)
double binom_cdf(uint32_t n, double p, uint32_t k)
{
    if (k >= n) return 1.0;
    double term = std::pow(1.0 - p, (double)n);   // P(X = 0)
    double acc = term;
    for (uint32_t i = 1; i <= k; i++) {
        term *= (double)(n - i + 1) / (double)i * p / (1.0 - p);
        acc += term;
    }
    return acc;
}

// ---------------------------------------------------------------------------
// jobs: launch and retire
// ---------------------------------------------------------------------------

void ensure_filter_operands(ifa_ctx *c);

// Launch arguments of a pass over chunk ch with the loaded queries, without
// the hit, work-list and counter fields.
// Strands per work item when a filter wave hands a whole batch to the
// resolve kernel (a wave holding an N). With few strands (one or two
// batches) such waves are most of the resolve kernel's work and the strands
// of an item run one after another in one resolve wave, so they are split
// finer to spread them over more waves.
uint32_t list_per(uint32_t n_sparse) { return n_sparse <= 64u ? 2u : 8u; }

ScanArgs chunk_args(ifa_ctx *c, const DevChunk &ch)
{
    ScanArgs a{};
    a.hi = ch.planes.p;
    a.lo = ch.planes.p + ch.stride;
    a.nm = ch.planes.p + 2 * ch.stride;
    a.em = ch.planes.p + 3 * ch.stride;
    a.nflag = ch.nflag.p;
    a.chunk_len = ch.len;
    a.own_from = ch.own_from;
    a.w_begin = 0;
    a.w_end = (uint32_t)((ch.len + 31) >> 5);
    a.lmax = c->lmax;
    a.qs = c->dq_qs;
    a.n_qs = (uint32_t)c->h_qs.size();
    a.n_sparse = c->n_sparse;
    a.policy = c->cfg.n_policy;
    a.list_per = list_per(a.n_sparse);
    a.qwords = c->dq_words;
    a.mq_b = c->dq_mqb;
    a.mq_t = c->dq_mqt;
    a.mq3_b = c->dq_mq3b;
    a.mq3_t = c->dq_mq3t;
    a.mq3_w = c->dq_mq3w;
    a.mq3_words = c->mq3_words;
    a.mq3_two_batches = c->mq3_two_batches;
    a.edge_pmin = c->edge_pmin;
    if (c->indexed) {
        a.seed_info = c->d_seed_info.p;
        a.seed_tab = c->d_seed_tab.p;
        a.seed_ncfg = (uint32_t)c->seeds.cfg.size();
        a.seed_mask = c->seedp.mask;
    }
    a.pieces = ch.pieces.p;
    a.n_pieces = ch.n_pieces;
    a.sink = c->cfg.sink;
    a.variant = c->variant;
    a.q_count = c->d_qcount.p;
    a.q_digest = c->d_qdigest.p;
    a.dm_first = a.n_qs;
    a.dense_seam = std::min<uint32_t>(std::max<uint32_t>(c->n_dm0, a.n_sparse), a.n_qs);
    a.dense_begin = a.n_sparse;
    a.dense_end = a.n_qs;
    a.dense_unclean = 0;
    uint32_t wpl, qu, wg, enc;
    variant_shape(c->variant, &wpl, &qu, &wg, &enc);
    if (enc == 3 && !c->indexed && c->n_dm0 < a.n_qs && c->dm_ready) {
        a.dm_first = c->n_dm0;
        a.dm_b = c->dq_dmb;
        a.dm_t = c->dq_dmt;
    }
    return a;
}

// Launch arguments of a pass over chunk ch into hit buffer hb (building the
// matrix filter's operands first if the variant needs new ones).
ScanArgs make_args(ifa_ctx *c, const DevChunk &ch, int hb)
{
    ensure_filter_operands(c);
    ScanArgs a = chunk_args(c, ch);
    a.work = c->work[hb].p;
    a.work_count = reinterpret_cast<unsigned int *>(c->d_ctr.p + 2 * hb + 1);
    a.skip_count = a.work_count + 1;
    a.work_cap = c->work_cap[hb];
    a.hits = c->d_hits[hb].p;
    a.hit_count = c->d_ctr.p + 2 * hb;
    a.hit_cap = c->buf_cap[hb];
    return a;
}

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
    return ms;
}

void collect_h2d_times(ifa_ctx *c)
{
    for (auto &pr : c->h2d_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(pr.second) == hipSuccess &&
            hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess)
            c->st.h2d_ms += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    c->h2d_pending.clear();
}

void copy_records(ifa_ctx *c, int hb, uint64_t n)
{
    if (n == 0) return;
    size_t old = c->hits.size();
    c->hits.resize(old + n);
    // the pass's done event has been waited on (it is recorded after the
    // pass, outside any graph); a copy on the compute stream would also wait
    // for the passes queued behind this one
    hip_check(hipMemcpy(c->hits.data() + old, c->d_hits[hb].p, n * sizeof(ifa_hit),
                        hipMemcpyDeviceToHost),
              "copy hit records");
    c->hits_sorted = false;
    c->st.hits += n;
}

// Timing events of one pass: t0 before the filter, t1 after it, td and tx
// before and after the dense kernels (on the stream they run on), te before
// the overhanging-window kernel, t2 after the last scan kernel.
struct PassEvents {
    hipEvent_t t0 = nullptr, t1 = nullptr, td = nullptr, tx = nullptr, te = nullptr,
               t2 = nullptr;
    void create()
    {
        if (!t0) hip_check(hipEventCreate(&t0), "event");
        if (!t1) hip_check(hipEventCreate(&t1), "event");
        if (!td) hip_check(hipEventCreate(&td), "event");
        if (!tx) hip_check(hipEventCreate(&tx), "event");
        if (!te) hip_check(hipEventCreate(&te), "event");
        if (!t2) hip_check(hipEventCreate(&t2), "event");
    }
    void destroy()
    {
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        if (td) (void)hipEventDestroy(td);
        if (tx) (void)hipEventDestroy(tx);
        if (te) (void)hipEventDestroy(te);
        if (t2) (void)hipEventDestroy(t2);
        t0 = t1 = td = tx = te = t2 = nullptr;
    }
};

// Does a pass over a (with its dense part if `dense`) run the dense kernels
// on the second stream?
bool forks(const ifa_ctx *c, const ScanArgs &a, bool dense)
{
    return c->overlap && !c->indexed && dense && a.n_sparse > 0 && a.n_sparse < a.n_qs;
}

// Enqueue one pass of the scan over a's word range: the sparse part (filter
// kernel, then resolve kernel over the work list) and, if `dense`, the dense
// kernels and (with IFA_FLAG_OVERHANG) the overhanging windows. Counters are
// cleared by kernels on the stream first. With both parts, the dense kernels
// run on the side stream, forked after the clear and joined before the
// overhanging windows, so that the device's workgroup slots are shared
// between the filter (mostly matrix-core work) and the dense kernels (vector
// ALU work) and neither's tail leaves it idle. They share only the pass
// counters and query sums, which both update atomically.
// (A null event in ev is not recorded.)
void enqueue_pass(ifa_ctx *c, const ScanArgs &a, bool clear_hits, bool dense, PassEvents &ev)
{
    auto mark = [&](hipEvent_t e, hipStream_t s) {
        if (e) hip_check(hipEventRecord(e, s), "event record");
    };
    // the pass counters of a hit buffer are adjacent (hit count, then the
    // work and skip counts): one clear kernel
    hip_check(clear_hits ? launch_clear_u64(a.hit_count, 2, c->comp_s)
                         : launch_clear_u64(a.hit_count + 1, 1, c->comp_s),
              "clear pass counters");
    hipStream_t cs = c->comp_s;
    mark(ev.t0, cs);
    if (c->indexed) {
        // indexed mode: seed lookups and their verification, one kernel
        mark(ev.t1, cs);
        mark(ev.td, cs);
        if (dense) hip_check(launch_seed(a, cs), "seed launch");
        mark(ev.tx, cs);
        mark(ev.te, cs);
        mark(ev.t2, cs);
        return;
    }
    const bool side = forks(c, a, dense);
    if (side) {
        hip_check(hipEventRecord(c->fork_ev, cs), "fork");
        hip_check(hipStreamWaitEvent(c->dense_s, c->fork_ev, 0), "fork");
        mark(ev.td, c->dense_s);
        hip_check(launch_dense(a, c->dense_s), "dense launch");
        mark(ev.tx, c->dense_s);
        hip_check(hipEventRecord(c->join_ev, c->dense_s), "join");
    }
    hip_check(launch_filter(a, cs), "filter launch");
    mark(ev.t1, cs);
    hip_check(launch_resolve(a, cs), "resolve launch");
    if (side) {
        hip_check(hipStreamWaitEvent(cs, c->join_ev, 0), "join");
    } else {
        mark(ev.td, cs);
        if (dense) hip_check(launch_dense(a, cs), "dense launch");
        mark(ev.tx, cs);
    }
    mark(ev.te, cs);
    if (dense && (c->cfg.flags & IFA_FLAG_OVERHANG))
        hip_check(launch_edge(a, cs), "overhang launch");
    mark(ev.t2, cs);
}

// The scan-kernel launches enqueue_pass issues for a (the clear kernel and
// events aside), in the same order.
std::vector<ScanLaunch> plan_pass(const ifa_ctx *c, const ScanArgs &a, bool dense)
{
    std::vector<ScanLaunch> p;
    if (c->indexed) {
        if (dense) hip_check(launch_seed(a, nullptr, &p), "plan");
        return p;
    }
    hip_check(launch_filter(a, nullptr, &p), "plan");
    hip_check(launch_resolve(a, nullptr, &p), "plan");
    if (dense) hip_check(launch_dense(a, nullptr, &p), "plan");
    if (dense && (c->cfg.flags & IFA_FLAG_OVERHANG)) hip_check(launch_edge(a, nullptr, &p), "plan");
    return p;
}

// Same kernels, blocks and LDS in the same order (grids and arguments may differ).
bool same_structure(const std::vector<ScanLaunch> &x, const std::vector<ScanLaunch> &y)
{
    if (x.size() != y.size()) return false;
    for (size_t i = 0; i < x.size(); i++)
        if (x[i].func != y[i].func || x[i].block.x != y[i].block.x || x[i].lds != y[i].lds)
            return false;
    return true;
}

// The scan-kernel nodes of a captured pass in plan order, or empty if the
// graph does not hold the plan. The graph is a chain, or (dense kernels on
// the side stream) a fork after the counter-clearing kernel into the filter
// and resolve kernels on one branch and the dense kernels on the other, then
// a join. Nodes are taken in dependency order; among the ready ones, the
// kernel the plan names next (the two branches launch different kernels).
std::vector<hipGraphNode_t> plan_kernel_nodes(hipGraph_t g, const std::vector<ScanLaunch> &plan)
{
    size_t n = 0;
    if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess) return {};
    std::vector<hipGraphNode_t> nodes(n);
    if (n && hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return {};
    std::map<hipGraphNode_t, size_t> pending;   // dependencies not yet taken
    std::vector<hipGraphNode_t> ready;
    for (hipGraphNode_t x : nodes) {
        size_t nd = 0;
        if (hipGraphNodeGetDependencies(x, nullptr, &nd) != hipSuccess) return {};
        pending[x] = nd;
        if (nd == 0) ready.push_back(x);
    }
    auto take = [&](size_t i) -> bool {
        hipGraphNode_t x = ready[i];
        ready.erase(ready.begin() + (std::ptrdiff_t)i);
        size_t nd = 0;
        if (hipGraphNodeGetDependentNodes(x, nullptr, &nd) != hipSuccess) return false;
        std::vector<hipGraphNode_t> dep(nd);
        if (nd && hipGraphNodeGetDependentNodes(x, dep.data(), &nd) != hipSuccess) return false;
        for (hipGraphNode_t y : dep)
            if (--pending[y] == 0) ready.push_back(y);
        return true;
    };
    std::vector<hipGraphNode_t> out;
    bool first = true;   // the counter-clearing kernel is not in the plan
    while (!ready.empty()) {
        bool moved = false;
        for (size_t i = 0; i < ready.size() && !moved; i++) {
            hipGraphNodeType t;
            if (hipGraphNodeGetType(ready[i], &t) != hipSuccess) return {};
            if (t != hipGraphNodeTypeKernel || first) {
                first = first && t != hipGraphNodeTypeKernel;
                if (!take(i)) return {};
                moved = true;
                continue;
            }
            hipKernelNodeParams kp{};
            if (hipGraphKernelNodeGetParams(ready[i], &kp) != hipSuccess) return {};
            if (out.size() < plan.size() && kp.func == plan[out.size()].func) {
                out.push_back(ready[i]);
                if (!take(i)) return {};
                moved = true;
            }
        }
        if (!moved) return {};
    }
    if (out.size() != plan.size()) return {};
    return out;
}

void enqueue_count_copies(ifa_ctx *c, int hb)
{
    hip_check(hipMemcpyAsync(c->h_ctr.p + 2 * hb, c->d_ctr.p + 2 * hb,
                             2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->comp_s),
              "copy pass counters");
}

// Pass counters of hit buffer hb on the host (valid after the pass's copy).
uint64_t host_hits(const ifa_ctx *c, int hb) { return c->h_ctr.p[2 * hb]; }
uint32_t host_work(const ifa_ctx *c, int hb)
{
    return reinterpret_cast<const unsigned int *>(c->h_ctr.p + 2 * hb + 1)[0];
}
uint32_t host_skip(const ifa_ctx *c, int hb)
{
    return reinterpret_cast<const unsigned int *>(c->h_ctr.p + 2 * hb + 1)[1];
}

// Book the times of a finished pass over words [w0, w1) whose counters are
// on the host. The filter evaluated every window start of the range except
// those of the waves it handed to the resolve kernel.
void add_pass_times(ifa_ctx *c, const PassEvents &ev, const Job &j, int hb, uint32_t w0,
                    uint32_t w1, bool split_timed)
{
    const bool sparse = j.args.n_sparse > 0;
    c->st.kernel_ms += elapsed(ev.t0, ev.t2);
    c->st.kernel_launches++;
    if (split_timed) {
        c->st.timed_passes++;
        if (c->cfg.flags & IFA_FLAG_OVERHANG) c->st.edge_ms += elapsed(ev.te, ev.t2);
        c->st.dense_ms += elapsed(ev.td, ev.tx);
        if (sparse) {
            c->st.filter_ms += elapsed(ev.t0, ev.t1);
            c->st.timed_filter_passes++;
        }
    }
    if (sparse) {
        c->st.filter_launches++;
        uint32_t wpl, qu, wg, enc;
        variant_shape(c->variant, &wpl, &qu, &wg, &enc);
        const uint64_t starts = 32ull * (w1 - w0);
        const uint64_t skipped = 64ull * wpl * host_skip(c, hb);
        const uint64_t evaluated = starts > skipped ? starts - skipped : 0;
        c->st.filter_windows += evaluated;
        c->st.filter_strand_windows += evaluated * j.args.n_sparse;
        c->st.filter_half_strand_windows += evaluated * j.n_half;
        c->st.work_items += host_work(c, hb);
    }
}

// A job's launch arguments with the hit buffer and work list of its hit
// buffer as they are now (either may have grown since the job was submitted).
ScanArgs job_args(const ifa_ctx *c, const Job &j)
{
    ScanArgs a = j.args;
    a.work = c->work[j.hitbuf].p;
    a.work_cap = c->work_cap[j.hitbuf];
    a.hits = c->d_hits[j.hitbuf].p;
    a.hit_cap = c->buf_cap[j.hitbuf];
    return a;
}

// Make the work list of hit buffer hb at least work_want items long (the
// list is not in use: its last pass has been retired).
void ensure_work_list(ifa_ctx *c, int hb)
{
    if (c->work_cap[hb] >= c->work_want) return;
    c->work[hb].alloc(c->work_want, "grow work list");
    c->work_cap[hb] = c->work_want;
}

// After a pass whose resolve kernel found the work list too small (and so
// did nothing), grow the list and run the sparse part again until it fits.
// Its dense part is not repeated: it does not use the list.
void settle_work_overflow(ifa_ctx *c, const Job &j, uint32_t w0, uint32_t w1)
{
    const int hb = j.hitbuf;
    while (host_work(c, hb) > c->work_cap[hb]) {
        const uint64_t need = (uint64_t)host_work(c, hb);
        const uint64_t cap = std::min<uint64_t>(need + need / 4 + 1024, 0xffffffffull);
        // the other list grows before its next launch: both see the same load
        c->work_want = std::max<uint32_t>(c->work_want, (uint32_t)cap);
        ensure_work_list(c, hb);
        ScanArgs a = job_args(c, j);
        a.w_begin = w0;
        a.w_end = w1;
        PassEvents ev;
        ev.create();
        enqueue_pass(c, a, false, false, ev);
        enqueue_count_copies(c, hb);
        hip_check(hipStreamSynchronize(c->comp_s), "sync");
        add_pass_times(c, ev, j, hb, w0, w1, true);
        ev.destroy();
        c->st.rescans++;
    }
}

// Re-scan word range [w0, w1) of a chunk whose hit buffer overflowed (the
// records of the first pass are discarded); halves the range until every
// part fits.
void rescan_range(ifa_ctx *c, const Job &j, uint32_t w0, uint32_t w1)
{
    const int hb = j.hitbuf;
    ScanArgs a = job_args(c, j);
    a.w_begin = w0;
    a.w_end = w1;
    PassEvents ev;
    ev.create();
    enqueue_pass(c, a, true, true, ev);
    enqueue_count_copies(c, hb);
    hip_check(hipStreamSynchronize(c->comp_s), "sync");
    add_pass_times(c, ev, j, hb, w0, w1, true);
    ev.destroy();
    c->st.rescans++;
    settle_work_overflow(c, j, w0, w1);
    uint64_t n = host_hits(c, hb);
    if (n <= c->buf_cap[hb]) {
        copy_records(c, hb, n);
        return;
    }
    if (w1 - w0 <= 1) {
        // one plane word holds 32 windows x every query strand; when those
        // alone overflow the buffer, the buffer grows to fit them
        c->d_hits[hb].alloc(n, "grow hit buffer");
        c->buf_cap[hb] = n;
        rescan_range(c, j, w0, w1);
        return;
    }
    uint32_t mid = w0 + (w1 - w0) / 2;
    rescan_range(c, j, w0, mid);
    rescan_range(c, j, mid, w1);
}

void retire(ifa_ctx *c, Job &j)
{
    if (!j.active) return;
    hip_check(hipEventSynchronize(j.done), "wait for scan");
    PassEvents ev;
    ev.t0 = j.k0;
    ev.t1 = j.kf;
    ev.td = j.kd;
    ev.tx = j.kx;
    ev.te = j.ke;
    ev.t2 = j.k1;
    const uint32_t words = (uint32_t)((j.chunk->len + 31) >> 5);
    add_pass_times(c, ev, j, j.hitbuf, 0, words, j.split_timed);
    settle_work_overflow(c, j, 0, words);
    if (c->cfg.sink == IFA_SINK_RECORDS) {
        uint64_t n = host_hits(c, j.hitbuf);
        if (n <= c->buf_cap[j.hitbuf]) {
            copy_records(c, j.hitbuf, n);
        } else {
            uint32_t mid = words / 2;
            rescan_range(c, j, 0, mid);
            rescan_range(c, j, mid, words);
        }
    }
    j.active = false;
}

void retire_all(ifa_ctx *c)
{
    // oldest first
    uint64_t s = c->job_seq;
    for (uint64_t i = (s >= 2 ? s - 2 : 0); i < s; i++) retire(c, c->jobs[i % 2]);
    collect_h2d_times(c);
}

// Launch the scan of a device chunk into the next hit buffer.
void submit_job(ifa_ctx *c, DevChunk *ch)
{
    Job &j = c->jobs[c->job_seq % 2];
    retire(c, j);   // frees the hit buffer and work list this job will use
    j.chunk = ch;
    j.hitbuf = (int)(c->job_seq % 2);
    ensure_work_list(c, j.hitbuf);
    ScanArgs a = make_args(c, *ch, j.hitbuf);
    j.args = a;
    {
        uint32_t wpl, qu, wg, enc;
        variant_shape(c->variant, &wpl, &qu, &wg, &enc);
        j.n_half = enc == 2 || enc == 3 ? c->n_half_strands : 0u;
    }
    if (!j.k0) hip_check(hipEventCreate(&j.k0), "event");
    if (!j.kf) hip_check(hipEventCreate(&j.kf), "event");
    if (!j.k1) hip_check(hipEventCreate(&j.k1), "event");
    if (!j.ke) hip_check(hipEventCreate(&j.ke), "event");
    if (!j.kd) hip_check(hipEventCreate(&j.kd), "event");
    if (!j.kx) hip_check(hipEventCreate(&j.kx), "event");
    if (!j.done) hip_check(hipEventCreateWithFlags(&j.done, hipEventDisableTiming), "event");
    PassEvents ev;
    ev.t0 = j.k0;
    ev.t1 = j.kf;
    ev.td = j.kd;
    ev.tx = j.kx;
    ev.te = j.ke;
    ev.t2 = j.k1;
    // the pass and its counter copy (what a graph holds). No event is
    // recorded inside a graph: a host wait on an event recorded by a graph
    // node has returned before a replay finished, and timing events recorded
    // by graph nodes read 10-15 % longer than the kernels between them
    // (against rocprofv3's kernel trace and the step's own wall time). A
    // replayed pass is timed as a whole by events around the graph launch;
    // its kernels are timed one by one only when launched eagerly.
    PassEvents none;
    auto enqueue = [&](PassEvents &e) {
        enqueue_pass(c, a, true, true, e);
        enqueue_count_copies(c, j.hitbuf);
    };
    PassGraph *pg = nullptr;
    std::vector<ScanLaunch> plan;
    if (c->cfg.flags & IFA_FLAG_GRAPHS) {
        pg = &ch->graph[j.hitbuf][c->tab];
        plan = plan_pass(c, a, true);
        if (!pg->seen || !same_structure(pg->plan, plan) || pg->forked != forks(c, a, true)) {
            // first pass of this structure: run eagerly, capture the next one
            pg->reset();
            pg->args = a;
            pg->plan = plan;
            pg->seen = true;
            pg->forked = forks(c, a, true);
            pg = nullptr;
        }
    }
    if (pg) {
        if (!pg->exec) {
            hip_check(hipStreamBeginCapture(c->comp_s, hipStreamCaptureModeRelaxed),
                      "begin capture");
            enqueue(none);
            hip_check(hipStreamEndCapture(c->comp_s, &pg->graph), "end capture");
            hip_check(hipGraphInstantiate(&pg->exec, pg->graph, nullptr, nullptr, 0),
                      "instantiate pass graph");
            pg->knodes = plan_kernel_nodes(pg->graph, plan);
            // a captured pass whose kernel nodes cannot be matched to its plan
            // could not be pointed at another chunk or query set later
            if (pg->knodes.size() != plan.size()) {
                pg->reset();
                fail(IFA_E_DEVICE, "pass graph layout");
            }
            pg->args = a;
            pg->plan = plan;
        } else if (std::memcmp(&pg->args, &a, sizeof a) != 0) {
            // another chunk or query set of the same structure: point the
            // captured kernels at it
            if (pg->knodes.size() != plan.size()) fail(IFA_E_DEVICE, "pass graph layout");
            for (size_t i = 0; i < plan.size(); i++) {
                hipKernelNodeParams kp{};
                void *kargs[] = {&plan[i].args};
                kp.func = const_cast<void *>(plan[i].func);
                kp.gridDim = plan[i].grid;
                kp.blockDim = plan[i].block;
                kp.sharedMemBytes = plan[i].lds;
                kp.kernelParams = kargs;
                kp.extra = nullptr;
                hip_check(hipGraphExecKernelNodeSetParams(pg->exec, pg->knodes[i], &kp),
                          "update pass graph");
            }
            pg->args = a;
            pg->plan = plan;
            c->st.graph_updates++;
        }
        hip_check(hipEventRecord(j.k0, c->comp_s), "event record");
        hip_check(hipGraphLaunch(pg->exec, c->comp_s), "launch pass graph");
        hip_check(hipEventRecord(j.k1, c->comp_s), "event record");
        c->st.graph_launches++;
        j.split_timed = false;
    } else {
        enqueue(ev);
        j.split_timed = true;
    }
    // a streamed chunk's slot may be refilled once this pass is done (the
    // copy stream waits for free_ev); resident chunks are never refilled
    if (!ch->resident) hip_check(hipEventRecord(ch->free_ev, c->comp_s), "event record");
    hip_check(hipEventRecord(j.done, c->comp_s), "event record");
    j.active = true;
    c->job_seq++;
    c->st.chunks++;
}

// Copy the hi and lo planes of a chunk's `used` words and its sparse list to
// device chunk d, then rebuild the nm and em planes, padding and N-block
// flags there, all on `stream`. The host buffers must stay untouched until
// the stream has passed this point.
void upload_planes(const uint32_t *hi, const uint32_t *lo, uint64_t used, const uint4 *list,
                   uint32_t n_list, DevChunk &d, hipStream_t stream)
{
    const uint64_t total = used + kPadWords;
    if (d.stride < total) fail(IFA_E_INVALID, "device chunk too small");
    if (d.nflag.n < nflag_blocks((uint32_t)d.stride))
        d.nflag.alloc(nflag_blocks((uint32_t)d.stride), "N-block flags");
    if (d.sparse.n < n_list) d.sparse.alloc(std::max<size_t>(n_list, 2 * d.sparse.n), "sparse list");
    hip_check(hipMemcpyAsync(d.planes.p, hi, used * sizeof(uint32_t), hipMemcpyHostToDevice,
                             stream),
              "copy hi plane");
    hip_check(hipMemcpyAsync(d.planes.p + d.stride, lo, used * sizeof(uint32_t),
                             hipMemcpyHostToDevice, stream),
              "copy lo plane");
    if (n_list)
        hip_check(hipMemcpyAsync(d.sparse.p, list, n_list * sizeof(uint4), hipMemcpyHostToDevice,
                                 stream),
                  "copy sparse list");
    hip_check(launch_expand(d.planes.p, d.stride, d.nflag.p, (uint32_t)used, (uint32_t)total,
                            d.sparse.p, n_list, stream),
              "expand chunk planes");
}

// Copy a sealed staging chunk into a device chunk on the copy stream.
void upload(ifa_ctx *c, Staging &s, DevChunk &d, hipStream_t stream)
{
    if (d.pieces.n < s.pieces.size() || d.pieces.p == nullptr)
        d.pieces.alloc(std::max<size_t>(s.pieces.size(), 1024), "device piece table");
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    hip_check(hipEventRecord(e0, stream), "event record");
    upload_planes(plane(c, s, 0), plane(c, s, 1), (s.len + 31) >> 5, s.list.p, s.n_list, d,
                  stream);
    if (!s.pieces.empty())
        hip_check(hipMemcpyAsync(d.pieces.p, s.pieces.data(), s.pieces.size() * sizeof(Piece),
                                 hipMemcpyHostToDevice, stream),
                  "copy piece table");
    hip_check(hipEventRecord(e1, stream), "event record");
    c->h2d_pending.emplace_back(e0, e1);
    d.len = s.len;
    d.own_from = s.own_from;
    d.n_pieces = (uint32_t)s.pieces.size();
}

void reset_staging(Staging &s)
{
    s.pieces.clear();
    s.tasks.clear();
    s.len = 0;
    s.own_from = 0;
    s.packed_to = 0;
}

void submit_staging(ifa_ctx *c);

// Submit the staging chunk being filled (if it holds any base) to the GPU.
void flush_stream(ifa_ctx *c)
{
    Staging &s = c->stage[c->cur];
    if (s.len == 0) {
        reset_staging(s);
        return;
    }
    pack_pending(c, s);
    seal(c, s);
    submit_staging(c);
}

// Upload the sealed staging chunk being filled to the next device slot, scan
// it, and switch to the other staging buffer.
void submit_staging(ifa_ctx *c)
{
    Staging &s = c->stage[c->cur];
    DevChunk &d = c->slot[c->chunk_seq % 2];
    // The device slot is reused. Its previous scan is retired first: an
    // overflowing hit buffer is re-scanned from this slot, so the slot must
    // not be overwritten before that job's hits are safe on the host.
    for (auto &j : c->jobs)
        if (j.active && j.chunk == &d) retire(c, j);
    hip_check(hipStreamWaitEvent(c->copy_s, d.free_ev, 0), "wait slot");
    upload(c, s, d, c->copy_s);
    hip_check(hipEventRecord(s.copied, c->copy_s), "event record");
    s.copy_pending = true;
    hip_check(hipStreamWaitEvent(c->comp_s, s.copied, 0), "wait copy");
    c->st.bases += s.len - s.own_from;
    submit_job(c, &d);
    c->chunk_seq++;
    // switch staging buffers; wait until the other one's copy has finished
    c->cur ^= 1;
    Staging &n = c->stage[c->cur];
    if (n.copy_pending) {
        hip_check(hipEventSynchronize(n.copied), "wait staging");
        n.copy_pending = false;
    }
    reset_staging(n);
}

// Append contigs to the chunk stream (or, when `sink` is given, to a
// sequence of chunks handed to `sink` as each one fills).
void append_contigs(ifa_ctx *c, uint32_t n_contigs, const uint8_t *const *seq,
                    const uint64_t *len, const std::function<void()> &on_full)
{
    const uint64_t cap = c->cfg.chunk_bases;
    for (uint32_t i = 0; i < n_contigs; i++) {
        const uint32_t ordinal = c->next_ordinal++;
        const uint64_t n = len[i];
        const uint8_t *src = seq[i];
        uint64_t x = 0;
        bool continuing = false;    // a piece of this contig is in an earlier chunk
        while (x < n) {
            Staging *s = &c->stage[c->cur];
            if (s->len == cap) {
                on_full();
                s = &c->stage[c->cur];
            }
            uint64_t carry = 0;
            if (continuing && s->len == 0) {
                carry = std::min<uint64_t>(kCarry, x);
                s->own_from = (uint32_t)carry;
            }
            uint64_t room = cap - s->len - carry;
            uint64_t take = std::min(room, n - x);
            Piece p{};
            p.start = s->len;
            p.len = carry + take;
            p.contig_off = x - carry;
            p.contig = ordinal;
            p.flags = (p.contig_off == 0 ? kPieceContigStart : 0u) |
                      (x + take == n ? kPieceContigEnd : 0u);
            s->pieces.push_back(p);
            s->tasks.push_back(PackTask{src + (x - carry), s->len, carry + take});
            s->len += carry + take;
            x += take;
            continuing = true;
        }
    }
}

// Prepare the device to run on the context's device in this thread.
void use_device(ifa_ctx *c) { hip_check(hipSetDevice(c->cfg.device), "hipSetDevice"); }

template <class F>
ifa_status guarded(ifa_ctx *c, F &&f)
{
    try {
        if (c) c->err.clear();
        f();
        return IFA_OK;
    } catch (const Failure &e) {
        if (c) c->err = e.msg;
        return e.st;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return IFA_E_NOMEM;
    } catch (...) {
        if (c) c->err = "unexpected internal error";
        return IFA_E_DEVICE;
    }
}

bool nothing_pending(ifa_ctx *c)
{
    if (c->stage[c->cur].len != 0) return false;
    for (auto &j : c->jobs)
        if (j.active) return false;
    return c->drain_pos >= c->hits.size();
}

// ---------------------------------------------------------------------------
// query tables
// ---------------------------------------------------------------------------

void validate_queries(uint32_t n, const uint8_t *const *seq, const uint32_t *len,
                      const int32_t *max_subs, const int32_t *max_n)
{
    if (n > 0 && (!seq || !len || !max_subs)) fail(IFA_E_INVALID, "NULL argument");
    for (uint32_t j = 0; j < n; j++) {
        if (len[j] == 0 || len[j] > IFA_MAX_QUERY_LEN)
            fail(IFA_E_TOO_LONG, "query " + std::to_string(j) + " has length " +
                                     std::to_string(len[j]) + " (allowed 1..255)");
        if (!seq[j]) fail(IFA_E_INVALID, "NULL query pointer");
        if (max_subs[j] < 0) fail(IFA_E_INVALID, "negative max_subs");
        if (max_n && max_n[j] < 0) fail(IFA_E_INVALID, "negative max_n");
    }
}

// Pack every selected strand of n queries into descriptors and plane words,
// appending to qs / words; query j gets qid qid_base + j. The offsets of every
// query's descriptors and words come first, then blocks of queries are packed
// on `threads` threads.
void pack_query_strands(uint32_t strands, uint32_t n, const uint8_t *const *seq,
                        const uint32_t *len, const int32_t *max_subs, const int32_t *max_n,
                        uint32_t qid_base, std::vector<QSDesc> &qs, std::vector<uint32_t> &words,
                        uint32_t &lmax, unsigned threads)
{
    const uint32_t ns = (strands & 1u) + ((strands >> 1) & 1u);
    const size_t q0 = qs.size();
    std::vector<size_t> woff(n + 1);
    woff[0] = words.size();
    for (uint32_t j = 0; j < n; j++) {
        lmax = std::max(lmax, len[j]);
        woff[j + 1] = woff[j] + (size_t)ns * 3u * ((len[j] + 31) / 32);
    }
    qs.resize(q0 + (size_t)ns * n);
    words.resize(woff[n], 0u);
    const size_t block = 1024;
    parallel_for(threads, (n + block - 1) / block, [&](size_t bi) {
        const uint32_t j1 = (uint32_t)std::min<size_t>(n, (bi + 1) * block);
        for (uint32_t j = (uint32_t)(bi * block); j < j1; j++) {
            const uint32_t L = len[j];
            uint8_t code[IFA_MAX_QUERY_LEN];
            for (uint32_t i = 0; i < L; i++) code[i] = kCode.c[seq[j][i]];
            uint32_t si = 0;
            for (uint32_t s = 0; s < 2; s++) {
                if (!(strands & (1u << s))) continue;
                QSDesc d{};
                d.qid = qid_base + j;
                d.len = (uint16_t)L;
                d.strand = (uint8_t)s;
                d.nw = (uint8_t)((L + 31) / 32);
                d.k = (uint16_t)std::min<int64_t>(max_subs[j], L);
                int64_t mn = max_n ? max_n[j] : (int64_t)(L / 4);
                d.maxn = (uint16_t)std::min<int64_t>(mn, L);
                d.woff = (uint32_t)(woff[j] + (size_t)si * 3u * d.nw);
                uint32_t *W = words.data() + d.woff;
                for (uint32_t i = 0; i < L; i++) {
                    // strand 1: reverse complement; complementing flips the hi
                    // bit of the code (A<->T, C<->G), N stays N
                    uint32_t v = s == 0 ? code[i] : code[L - 1 - i];
                    if (s == 1 && v < 4) v ^= 2u;
                    uint32_t t = i >> 5, bit = 1u << (i & 31);
                    if (v == 4) {
                        W[3 * t + 2] |= bit;
                    } else {
                        if (v & 2) W[3 * t] |= bit;
                        if (v & 1) W[3 * t + 1] |= bit;
                    }
                }
                d.qh0 = W[0];
                d.ql0 = W[1];
                d.qn0 = W[2];
                // the filter counts mismatches over the first min(L, 32) bases
                d.thr = d.k;
                qs[q0 + (size_t)ns * j + si] = d;
                si++;
            }
        }
    });
}

// Make qs / words the context's query table. Partition: strands whose filter
// is expected to pass a window in 1/32 of the waves or more (filter_words) are
// dense and skip the filter's work list. Sparse strands go first, then dense ones; each group sorted by L
// descending (the kernels mask their cached slices in place as L drops),
// then by k. n_queries sizes the
// count+digest accumulators, which this resets.
// The first K step of a one-word three-class tile holds the 8-base blocks 0
// and 1 of each group's segment in all three classes (and block 2 in two),
// so on its own it tests the window at shift r (0..7) of a group on the
// strand's first min(L, 16 - r) bases. A tile whose strands all pass a
// 1024-window wave that way less than kHalfWaveRate of the time runs that
// step alone (half the matrix work; maxSubs 0 qualifies from L = 16 on).
constexpr double kHalfWaveRate = 1.0 / 1024.0;

// Dense strands the encoding-3 variants count on the matrix cores (on clean
// waves): at most 32 bases, so that one prefix word holds the whole strand,
// and a random window hit rate of at most kDenseMatrixRate, so that their
// hits, listed per accumulator register, stay few. The others (short strands
// with high maxSubs) stay on the VALU kernels, whose hit list serves every
// lane when nearly every window hits. (On 10,000 queries of 18-50 bases with
// maxSubs 0-16, limits of 0.02 and 0.2 gave 1 % and 4 % slower passes.)
constexpr double kDenseMatrixRate = 0.05;

bool dense_matrix_ok(const QSDesc &d)
{
    return d.len <= 32u && binom_cdf(d.len, 0.75, d.k) <= kDenseMatrixRate;
}

// Mean over the 8 shifts of P(a random window passes the half-step filter).
double half_step_rate(const QSDesc &d)
{
    const uint32_t lf = std::min<uint32_t>(d.len, 32u);
    double p = 0.0;
    for (uint32_t r = 0; r < 8; r++) p += binom_cdf(std::min<uint32_t>(lf, 16u - r), 0.75, d.thr);
    return p / 8.0;
}

bool half_step_ok(const QSDesc &d, uint8_t fw)
{
    return fw == 1 && half_step_rate(d) * 1024.0 < kHalfWaveRate;
}

// P(a random window passes the strand's filter): on its first
// min(L, 32 fw) bases, or the half step.
double window_pass_rate(const QSDesc &d, uint8_t fw, bool half)
{
    if (half) return half_step_rate(d);
    const uint32_t lf = std::min<uint32_t>(d.len, 32u * std::max<uint32_t>(fw, 1u));
    return binom_cdf(lf, 0.75, d.thr);
}

// Expected work items the filter emits per chunk of chunk_bases uniform
// random bases, for sparse strands qs[0, n_sparse): an item is one (wave,
// batch of 32 strands) with a candidate among the wave's windows (64 lanes x
// at most 16 windows); waves holding a reference N add items of their own,
// for which the list grows when they are many.
uint64_t expected_work_items(const std::vector<QSDesc> &qs, const std::vector<uint8_t> &fw,
                             uint32_t n_sparse, uint64_t chunk_bases)
{
    const double waves = (double)chunk_bases / 1024.0 + 1.0;
    double items = 0.0;
    for (uint32_t b = 0; b < n_sparse; b += 32) {
        double log_none = 0.0;
        for (uint32_t s = b; s < std::min<uint32_t>(n_sparse, b + 32); s++) {
            const double p = window_pass_rate(qs[s], fw[s], half_step_ok(qs[s], fw[s]));
            log_none += 1024.0 * std::log1p(-std::min(p, 1.0 - 1e-12));
        }
        items += waves * -std::expm1(log_none);
    }
    return (uint64_t)(items * 1.5);
}

// Operands of the matrix-core filter for sparse strands qs[0, n_sparse): tile
// nt holds strands 2nt and 2nt+1, column c = 16 (strand - 2nt) + shift r. The
// B operand of K step t for lane l (column l % 32, half h = l / 32) has in
// register b, nibble o the e2m1 value 1.0 (code 2) when the strand's base at
// j = 16t + 8h + o - r exists (0 <= j < min(L, 32)), is not N and has code b
// (= 2 hi + lo), else 0. need[c] = min(L, 32) - thr: the matches a window
// must reach to remain a candidate (filter count <= thr).
void build_mfma_operands(const std::vector<QSDesc> &qs, uint32_t n_sparse,
                         std::vector<uint32_t> &b, std::vector<float> &need, unsigned threads)
{
    const uint32_t n_tiles = (n_sparse + 1) / 2;
    b.assign((size_t)n_tiles * 3 * 64 * 4, 0u);
    need.assign((size_t)n_tiles * 32, 1e30f);
    const uint32_t block = 4096;
    parallel_for(threads, (n_tiles + block - 1) / block, [&](size_t bi) {
    const uint32_t nt1 = (uint32_t)std::min<size_t>(n_tiles, (bi + 1) * block);
    for (uint32_t nt = (uint32_t)(bi * block); nt < nt1; nt++) {
        for (uint32_t c = 0; c < 32; c++) {
            const uint32_t s = 2 * nt + c / 16, r = c % 16;
            if (s >= n_sparse) continue;
            const QSDesc &d = qs[s];
            const uint32_t l32 = std::min<uint32_t>(d.len, 32u);
            need[32 * nt + c] = (float)l32 - (float)d.thr;
            for (uint32_t t = 0; t < 3; t++)
                for (uint32_t h = 0; h < 2; h++)
                    for (uint32_t o = 0; o < 8; o++) {
                        const int32_t j = (int32_t)(16 * t + 8 * h + o) - (int32_t)r;
                        if (j < 0 || j >= (int32_t)l32 || ((d.qn0 >> j) & 1u)) continue;
                        const uint32_t cls = 2u * ((d.qh0 >> j) & 1u) + ((d.ql0 >> j) & 1u);
                        const size_t lane = c + 32 * h;
                        b[((3 * (size_t)nt + t) * 64 + lane) * 4 + cls] |= 2u << (4 * o);
                    }
        }
    }
    });
}

// Longest filter prefix, in 32-base words (the three-class matrix filter
// reads up to this many; the other filters read one).
constexpr uint32_t kFilterWords = 2;

// Operands of the three-class matrix-core filter: tile nt holds strands
// 4nt .. 4nt+3, column c = 8 (strand - 4nt) + shift r, and filters on the
// first Lf = min(L, 32 W) bases of each, W = words[nt] & 0xff = the most
// prefix words (filter_words) any of its strands needs; a half-step tile
// (words[nt] & kHalfTile) on the first Lt = min(Lf, 16 - r) only, else Lt =
// Lf. For word w < W, lane l (column l % 32, half h = l / 32), K step t,
// register d the slot is z = 8t + 4h + d: segment block k = z / 3 and class
// z % 3 (C, G, T; codes 1, 3, 2); nibble o is segment base i = 8k + o and
// query base j = 32w + i - r. The value is +1.0 (e2m1 code 2) when 32w <= j <
// min(32(w + 1), Lt) and the query base there has the slot's class, -1.0
// (code 0xA) when it is A, else 0; slot 15 stays 0. Layout:
// b[(((2 nt + w) * 2 + t) * 64 + lane) * 4 + d] (word 1 is zero when W = 1).
// need[c] = Lt - thr - nA, nA = A bases among the first Lt.
// Prefix words of each three-class column tile: the most any of its strands needs.
void mfma3_tile_words(const std::vector<uint8_t> &fw, uint32_t n_sparse,
                      std::vector<uint32_t> &words)
{
    const uint32_t n_tiles = (n_sparse + 3) / 4;
    words.assign(n_tiles, 1u);
    for (uint32_t nt = 0; nt < n_tiles; nt++)
        for (uint32_t s = 4 * nt; s < std::min(n_sparse, 4 * nt + 4); s++)
            words[nt] = std::max<uint32_t>(words[nt], fw[s]);
}

// Per three-class column tile of the sparse strands: the prefix words it
// filters on, plus kHalfTile when every strand of the tile qualifies for the
// half step (see half_step_ok).
constexpr uint32_t kHalfTile = 0x100u;

void mfma3_tile_meta(const std::vector<QSDesc> &qs, const std::vector<uint8_t> &fw,
                     uint32_t n_sparse, std::vector<uint32_t> &meta)
{
    mfma3_tile_words(fw, n_sparse, meta);
    for (uint32_t nt = 0; nt < meta.size(); nt++) {
        bool half = meta[nt] == 1u;
        for (uint32_t s = 4 * nt; half && s < std::min(n_sparse, 4 * nt + 4); s++)
            half = half_step_ok(qs[s], fw[s]);
        if (half) meta[nt] |= kHalfTile;
    }
}

void build_mfma3_operands(const std::vector<QSDesc> &qs, const std::vector<uint32_t> &qw,
                          const std::vector<uint32_t> &words, uint32_t n_sparse,
                          std::vector<uint32_t> &b, std::vector<float> &need, unsigned threads)
{
    static const uint32_t kClass[3] = {1u, 3u, 2u};
    const uint32_t n_tiles = (n_sparse + 3) / 4;
    b.assign((size_t)n_tiles * kFilterWords * 2 * 64 * 4, 0u);
    need.assign((size_t)n_tiles * 32, 1e30f);
    const uint32_t block = 2048;
    parallel_for(threads, (n_tiles + block - 1) / block, [&](size_t bi) {
    const uint32_t nt1 = (uint32_t)std::min<size_t>(n_tiles, (bi + 1) * block);
    for (uint32_t nt = (uint32_t)(bi * block); nt < nt1; nt++) {
        for (uint32_t c = 0; c < 32; c++) {
            const uint32_t s = 4 * nt + c / 8, r = c % 8;
            if (s >= n_sparse) continue;
            const QSDesc &d = qs[s];
            const bool half = (words[nt] & kHalfTile) != 0u;
            const uint32_t nw = words[nt] & 0xffu;
            const uint32_t lf = std::min<uint32_t>(d.len, 32u * nw);
            // bases the column tests: a half-step column at shift r only its
            // first min(lf, 16 - r)
            const uint32_t lt = half ? std::min<uint32_t>(lf, 16u - r) : lf;
            // the strand's bases 0 .. lf-1 (lf <= 64) from its packed words
            uint8_t code[64], isn[64];
            for (uint32_t j = 0; j < lf; j++) {
                const uint32_t wd = j >> 5, bit = j & 31;
                const uint32_t qh = wd == 0 ? d.qh0 : qw[d.woff + 3 * wd];
                const uint32_t ql = wd == 0 ? d.ql0 : qw[d.woff + 3 * wd + 1];
                const uint32_t qn = wd == 0 ? d.qn0 : qw[d.woff + 3 * wd + 2];
                code[j] = (uint8_t)(2u * ((qh >> bit) & 1u) + ((ql >> bit) & 1u));
                isn[j] = (uint8_t)((qn >> bit) & 1u);
            }
            uint32_t n_a = 0;
            for (uint32_t j = 0; j < lt; j++)
                if (!isn[j] && code[j] == 0u) n_a++;
            need[32 * nt + c] = (float)lt - (float)d.thr - (float)n_a;
            for (uint32_t w = 0; w < nw; w++)
                for (uint32_t h = 0; h < 2; h++)
                    for (uint32_t t = 0; t < 2; t++)
                        for (uint32_t dd = 0; dd < 4; dd++) {
                            // K step t holds slots 8t .. 8t + 7, lane half h
                            // four of them
                            const uint32_t z = 8 * t + 4 * h + dd;
                            if (z >= 15) continue;
                            const uint32_t k = z / 3, cls = kClass[z % 3];
                            uint32_t word = 0;
                            for (uint32_t o = 0; o < 8; o++) {
                                const int32_t j = (int32_t)(32 * w + 8 * k + o) - (int32_t)r;
                                if (j < (int32_t)(32 * w) || j >= (int32_t)std::min(32 * w + 32, lt))
                                    continue;
                                if (isn[j]) continue;
                                if (code[j] == cls) word |= 0x2u << (4 * o);
                                else if (code[j] == 0u) word |= 0xAu << (4 * o);
                            }
                            const size_t lane = c + 32 * h;
                            b[((((size_t)nt * kFilterWords + w) * 2 + t) * 64 + lane) * 4 + dd] = word;
                        }
        }
    }
    });
}

// 32-base words of the strand's prefix a filter needs so that it passes a
// window in under 1/32 of the 1024-window waves on iid bases (P(Bin(Lf, 3/4)
// <= thr) * 1024 < 1/32 with Lf = min(L, 32 w)), for w up to kFilterWords;
// 0 when no such prefix exists (the strand is dense). Strands that pass more
// often cost less in the dense kernels than as work items: on the batched
// 10,000-query workload the bound 1/32 ran 19 % faster than 1/2 (1/8 to
// 1/128 within 2 % of it).
constexpr double kSparseWaveRate = 1.0 / 32.0;

uint32_t filter_words(const QSDesc &d)
{
    for (uint32_t w = 1; w <= kFilterWords; w++) {
        const uint32_t lf = std::min<uint32_t>(d.len, 32u * w);
        if (d.thr < lf && binom_cdf(lf, 0.75, d.thr) * 1024.0 < kSparseWaveRate) return w;
        if (lf == d.len) break;
    }
    return 0;
}

// One part of a table upload: parts go at 256-byte offsets of one arena.
struct TablePart {
    const void *src;
    size_t bytes;
};

// Copy `n` parts through the pinned staging `h` into the device arena `d`
// (both grown as needed) with one copy on the compute stream, after the work
// already queued there; off[i] gets part i's offset. `staged` marks the end
// of the staging's last copy: it is waited for before the staging is
// rewritten, and recorded again after this copy. Returns the arena.
uint8_t *upload_tables(ifa_ctx *c, HostBuf<uint8_t> &h, DevBuf<uint8_t> &d, const TablePart *parts,
                       int n, size_t *off, const char *what, hipEvent_t &staged)
{
    size_t total = 0;
    for (int i = 0; i < n; i++) {
        off[i] = total;
        total += (std::max<size_t>(parts[i].bytes, 16) + 255) & ~(size_t)255;
    }
    if (staged) hip_check(hipEventSynchronize(staged), "wait for table staging");
    else hip_check(hipEventCreateWithFlags(&staged, hipEventDisableTiming), "event");
    if (h.n < total) h.alloc(total, "pinned table staging");
    if (d.n < total) {
        // queued passes may still read the arena being replaced
        hip_check(hipStreamSynchronize(c->comp_s), "sync");
        d.alloc(total, what);
    }
    for (int i = 0; i < n; i++)
        if (parts[i].bytes) std::memcpy(h.p + off[i], parts[i].src, parts[i].bytes);
    hip_check(hipMemcpyAsync(d.p, h.p, total, hipMemcpyHostToDevice, c->comp_s), what);
    hip_check(hipEventRecord(staged, c->comp_s), "event record");
    return d.p;
}

// The B operands and required counts of the matrix-core filter form a
// variant uses, for the loaded query set: form 0 (four-class, encoding 1) or
// 1 (three-class, encodings 2 and 3; with encoding 3 also the one-word
// operands of the dense strands of at most 32 bases).
struct FilterOperands {
    int form = -1;            // -1: the variant needs none
    bool dense = false;
    std::vector<uint32_t> b, db;
    std::vector<float> need, dneed;
};

FilterOperands build_filter_operands(const ifa_ctx *c)
{
    FilterOperands op;
    if (c->indexed) return op;
    uint32_t wpl, qu, wg, enc;
    variant_shape(c->variant, &wpl, &qu, &wg, &enc);
    if (enc < 1 || enc > 3) return op;
    const uint32_t n_qs = (uint32_t)c->h_qs.size();
    const bool dense = enc == 3 && c->n_dm0 < n_qs;
    if (c->n_sparse == 0 && !dense) return op;
    const int f = enc == 1 ? 0 : 1;
    if (c->mq_ready[f] && (!dense || c->dm_ready)) return op;
    op.form = f;
    op.dense = dense;
    if (enc == 1) {
        build_mfma_operands(c->h_qs, c->n_sparse, op.b, op.need, c->threads);
    } else {
        std::vector<uint32_t> mw3;
        mfma3_tile_meta(c->h_qs, c->h_fw, c->n_sparse, mw3);
        build_mfma3_operands(c->h_qs, c->h_qwords, mw3, c->n_sparse, op.b, op.need, c->threads);
        if (dense) {
            // the dense strands of at most 32 bases: one-word tiles, their
            // bound the exact hit test (thr = k)
            std::vector<QSDesc> dq(c->h_qs.begin() + c->n_dm0, c->h_qs.end());
            std::vector<uint32_t> one((dq.size() + 3) / 4, 1u);
            std::vector<uint32_t> db;
            build_mfma3_operands(dq, c->h_qwords, one, (uint32_t)dq.size(), db, op.dneed,
                                 c->threads);
            // keep only the first word's operands of each tile (2 K steps)
            op.db.reserve(one.size() * 2 * 64 * 4);
            for (size_t nt = 0; nt < one.size(); nt++) {
                const size_t base = nt * kFilterWords * 2 * 64 * 4;
                op.db.insert(op.db.end(), db.begin() + base, db.begin() + base + 2 * 64 * 4);
            }
        }
    }
    return op;
}

// The four upload parts of op (operands, counts, dense operands, dense counts).
void filter_operand_parts(const FilterOperands &op, TablePart *parts)
{
    parts[0] = {op.b.data(), op.b.size() * sizeof(uint32_t)};
    parts[1] = {op.need.data(), op.need.size() * sizeof(float)};
    parts[2] = {op.db.data(), op.db.size() * sizeof(uint32_t)};
    parts[3] = {op.dneed.data(), op.dneed.size() * sizeof(float)};
}

// Point the context at operands uploaded to base + off[0..3].
void set_filter_operands(ifa_ctx *c, const FilterOperands &op, const uint8_t *base,
                         const size_t *off)
{
    if (op.form == 0) {
        c->dq_mqb = reinterpret_cast<const uint4 *>(base + off[0]);
        c->dq_mqt = reinterpret_cast<const float *>(base + off[1]);
    } else {
        c->dq_mq3b = reinterpret_cast<const uint4 *>(base + off[0]);
        c->dq_mq3t = reinterpret_cast<const float *>(base + off[1]);
        c->dq_dmb = reinterpret_cast<const uint4 *>(base + off[2]);
        c->dq_dmt = reinterpret_cast<const float *>(base + off[3]);
        c->dm_ready = op.dense;
    }
    c->mq_ready[op.form] = true;
}

// Build and upload the matrix-core filter operands of the context's variant
// if the loaded query set does not have them yet (the variant changed after
// the queries were loaded; install_queries uploads those of the variant in
// use with the query tables).
void ensure_filter_operands(ifa_ctx *c)
{
    if (!c->have_queries) return;
    const FilterOperands op = build_filter_operands(c);
    if (op.form < 0) return;
    TablePart parts[4];
    filter_operand_parts(op, parts);
    size_t off[4];
    const int t = c->tab;
    const uint8_t *base = upload_tables(c, c->h_mqarena[t][op.form], c->d_mqarena[t][op.form],
                                        parts, 4, off, "matrix filter operands",
                                        c->mqstaged[t][op.form]);
    set_filter_operands(c, op, base, off);
}

void install_queries(ifa_ctx *c, std::vector<QSDesc> &&qs, std::vector<uint32_t> &&words,
                     uint32_t n_queries, uint32_t lmax)
{
    const bool indexed = c->indexed;
    std::vector<uint8_t> fw(qs.size()), dense(qs.size()), dm(qs.size());
    for (size_t i = 0; i < qs.size(); i++) {
        fw[i] = (uint8_t)filter_words(qs[i]);
        dense[i] = fw[i] == 0;
        dm[i] = dense[i] && !indexed && dense_matrix_ok(qs[i]);
    }
    std::vector<size_t> order(qs.size());
    for (size_t i = 0; i < order.size(); i++) order[i] = i;
    // sparse strands filtered on two words first (all have L > 32, so min(L,
    // 32) still never rises along the list), then L descending, then k; the
    // dense strands the matrix cores may count last among the dense ones
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        if (dense[x] != dense[y]) return dense[x] < dense[y];
        if (dm[x] != dm[y]) return dm[x] < dm[y];
        if (fw[x] != fw[y]) return fw[x] > fw[y];
        const QSDesc &a = qs[x], &b = qs[y];
        if (a.len != b.len) return a.len > b.len;
        return a.k < b.k;
    });
    std::vector<QSDesc> sorted;
    std::vector<uint8_t> sorted_fw;
    sorted.reserve(qs.size());
    uint32_t n_sparse = 0;
    for (size_t i : order) {
        sorted.push_back(qs[i]);
        sorted_fw.push_back(fw[i]);
        if (!dense[i]) n_sparse++;
    }
    qs.swap(sorted);
    std::vector<uint32_t> mw3;
    if (!indexed) mfma3_tile_meta(qs, sorted_fw, n_sparse, mw3);
    c->mq3_words = 1;
    for (uint32_t m : mw3) c->mq3_words = std::max(c->mq3_words, m & 0xffu);
    // the tiles filtering on two words lead the list: their batches of 32
    // strands (8 tiles) run the two-word kernel, the others the one-word one
    uint32_t two_tiles = 0;
    while (two_tiles < mw3.size() && (mw3[two_tiles] & 0xffu) == 2u) two_tiles++;
    c->mq3_two_batches = (two_tiles + 7u) / 8u;
    c->n_half_strands = 0;
    for (uint32_t nt = 0; nt < mw3.size(); nt++)
        if (mw3[nt] & kHalfTile) c->n_half_strands += std::min<uint32_t>(4u, n_sparse - 4u * nt);
    // overhang kernel packing: 2 C window slots per piece and strand, C =
    // min(maxN, L - 1); the widest clip sets the pieces per wave of the grid
    uint32_t cmax = 0;
    for (const QSDesc &d : qs) cmax = std::max<uint32_t>(cmax, std::min<uint32_t>(d.maxn, d.len - 1u));
    c->edge_pmin = cmax == 0 ? 0u : (2u * cmax <= 64u ? 64u / (2u * cmax) : 1u);
    uint32_t n_dm0 = n_sparse;
    for (size_t i : order)
        if (dense[i] && !dm[i]) n_dm0++;
    c->n_dm0 = n_dm0;   // [n_dm0, size): the matrix-counted dense strands
    if (c->cfg.work_capacity == 0 && !indexed) {
        // size the work lists for the expected load unless the caller fixed
        // the initial capacity (they grow on overflow either way)
        const uint64_t est = expected_work_items(qs, sorted_fw, n_sparse, c->cfg.chunk_bases);
        c->work_want =
            (uint32_t)std::min<uint64_t>(std::max<uint64_t>(est, c->work_want), 1ull << 28);
    }
    c->h_qs = std::move(qs);
    c->h_fw = std::move(sorted_fw);
    c->n_sparse = n_sparse;
    c->h_qwords = std::move(words);
    c->n_queries = n_queries;
    c->lmax = std::max<uint32_t>(lmax, 1);
    c->have_queries = false;   // until the tables are on the device
    c->mq_ready[0] = c->mq_ready[1] = false;
    c->dm_ready = false;
    // one upload of every table, the variant's filter operands included:
    // parts at 256-byte offsets in one arena
    const FilterOperands op = build_filter_operands(c);
    TablePart parts[7] = {{c->h_qs.data(), c->h_qs.size() * sizeof(QSDesc)},
                          {c->h_qwords.data(), c->h_qwords.size() * sizeof(uint32_t)},
                          {mw3.data(), mw3.size() * sizeof(uint32_t)}};
    const int n_parts = op.form < 0 ? 3 : 7;
    if (op.form >= 0) filter_operand_parts(op, parts + 3);
    size_t off[7];
    c->tab ^= 1;
    const uint8_t *base = upload_tables(c, c->h_qarena[c->tab], c->d_qarena[c->tab], parts,
                                        n_parts, off, "query tables", c->qstaged[c->tab]);
    c->dq_qs = reinterpret_cast<const QSDesc *>(base + off[0]);
    c->dq_words = reinterpret_cast<const uint32_t *>(base + off[1]);
    c->dq_mq3w = reinterpret_cast<const uint32_t *>(base + off[2]);
    if (op.form >= 0) set_filter_operands(c, op, base, off + 3);
    if (c->cfg.sink == IFA_SINK_COUNT_DIGEST) {
        const size_t need = (size_t)std::max<uint32_t>(n_queries, 1) * kStripes;
        if (c->d_qcount.n < need) {
            c->d_qcount.alloc(need, "query counters");
            c->d_qdigest.alloc(need, "query digests");
        }
        hip_check(launch_clear_u64(c->d_qcount.p, (uint32_t)need, c->comp_s), "clear counters");
        hip_check(launch_clear_u64(c->d_qdigest.p, (uint32_t)need, c->comp_s), "clear digests");
    }
    c->hits.clear();
    c->drain_pos = 0;
    c->hits_sorted = true;
    c->have_queries = true;
}

// Indexed mode: seeds of the query set just installed (c->h_qs, device
// order) and their device tables.
void install_seeds(ifa_ctx *c, uint32_t n, const uint32_t *len, const int32_t *max_subs,
                   const uint8_t *const *seq, const int32_t *max_n)
{
    // the query set is unusable until its seed tables match it
    c->have_queries = false;
    // every query's forward strand, packed like the strands
    std::vector<QSDesc> fq;
    std::vector<uint32_t> fw, foff(n);
    uint32_t lmax = 0;
    pack_query_strands(1u, n, seq, len, max_subs, max_n, 0, fq, fw, lmax, c->threads);
    for (uint32_t j = 0; j < n; j++) foff[j] = fq[j].woff;
    SeedBuild b;
    build_seeds(c->seedp, n, len, max_subs, c->h_qs, c->h_qwords, fw, foff, c->threads,
                c->mh_cache, b);
    if (b.cfg.size() > kMaxSeedCfg) fail(IFA_E_INVALID, "more than 8 distinct seed lengths");
    // uploads are ordered on the compute stream (the stream does not wait for
    // the null stream) and complete before the host tables are released
    hip_check(hipStreamSynchronize(c->comp_s), "sync");
    // buffers grow only, so repeated query sets of the same shape keep their
    // device addresses (and their captured pass graphs)
    if (c->d_seed_info.n < std::max<size_t>(b.info.size(), 1))
        c->d_seed_info.alloc(std::max<size_t>(b.info.size(), 1), "seed info");
    if (!b.info.empty())
        hip_check(hipMemcpyAsync(c->d_seed_info.p, b.info.data(),
                                 b.info.size() * sizeof(SeedInfo), hipMemcpyHostToDevice,
                                 c->comp_s),
                  "upload seed info");
    for (size_t i = 0; i < kMaxSeedCfg; i++) {
        if (i >= b.cfg.size()) continue;
        const SeedBuild::Cfg &g = b.cfg[i];
        if (c->d_seed_dir[i].n < g.dir.size()) c->d_seed_dir[i].alloc(g.dir.size(), "seed directory");
        if (c->d_seed_ent[i].n < std::max<size_t>(g.ent.size(), 2))
            c->d_seed_ent[i].alloc(std::max<size_t>(g.ent.size(), 2), "seed entries");
        hip_check(hipMemcpyAsync(c->d_seed_dir[i].p, g.dir.data(),
                                 g.dir.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                 c->comp_s),
                  "upload seed directory");
        if (!g.ent.empty())
            hip_check(hipMemcpyAsync(c->d_seed_ent[i].p, g.ent.data(),
                                     g.ent.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                                     c->comp_s),
                      "upload seed entries");
    }
    SeedTable tab[kMaxSeedCfg] = {};
    for (size_t i = 0; i < b.cfg.size(); i++) {
        tab[i].k = b.cfg[i].k;
        tab[i].bits = b.cfg[i].bits;
        tab[i].dir = c->d_seed_dir[i].p;
        tab[i].ent = reinterpret_cast<const uint2 *>(c->d_seed_ent[i].p);
        // presence bitmap, built on the device from the uploaded entries
        const uint32_t key_bits = 2u * (b.cfg[i].k - c->seedp.mask);
        const size_t words = std::max<size_t>(1, ((size_t)1 << seed_bitmap_bits(key_bits)) / 32);
        if (c->d_seed_bm[i].n < words) c->d_seed_bm[i].alloc(words, "seed presence bitmap");
        hip_check(launch_seed_bitmap(tab[i].ent, (uint32_t)(b.cfg[i].ent.size() / 2),
                                     c->d_seed_bm[i].p, (uint32_t)words, key_bits, c->comp_s),
                  "seed presence bitmap");
        tab[i].bm = c->d_seed_bm[i].p;
        tab[i].key_bits = key_bits;
    }
    if (!c->d_seed_tab.p) c->d_seed_tab.alloc(kMaxSeedCfg, "seed table descriptors");
    hip_check(hipMemcpyAsync(c->d_seed_tab.p, tab, sizeof tab, hipMemcpyHostToDevice, c->comp_s),
              "upload seed table descriptors");
    hip_check(hipStreamSynchronize(c->comp_s), "sync seed uploads");
    c->seeds = std::move(b);
    c->have_queries = true;
}

// Autotune cache key: device architecture, query-strand count band (log2),
// longest query in words, threshold band. Tile choice depends on these.
std::string tune_key(ifa_ctx *c)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->cfg.device) == hipSuccess) arch = prop.gcnArchName;
    for (auto &ch : arch)
        if (ch == ' ' || ch == '\t') ch = '_';
    uint32_t nqs = (uint32_t)c->h_qs.size(), band = 0;
    while ((1u << band) < nqs) band++;
    uint32_t nw = 0, kmin = 0xffff, kmax = 0;
    for (const QSDesc &d : c->h_qs) {
        nw = std::max<uint32_t>(nw, d.nw);
        kmin = std::min<uint32_t>(kmin, d.k);
        kmax = std::max<uint32_t>(kmax, d.k);
    }
    return arch + "|q2^" + std::to_string(band) + "|w" + std::to_string(nw) + "|k" +
           std::to_string(kmin / 4) + "-" + std::to_string(kmax / 4) + "|v" +
           std::to_string(ifa::variant_count()) + (c->overlap ? "|o" : "");
}

bool cache_lookup(const char *path, const std::string &key, uint32_t *v)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[400];
        unsigned vv;
        double ms;
        if (std::sscanf(line, "%399s %u %lf", k, &vv, &ms) == 3 && key == k) {
            *v = vv;
            found = true;   // the last entry for a key wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, uint32_t v, double ms)
{
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %u %.6f\n", key.c_str(), v, ms);
    std::fclose(f);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

namespace {

// A pass of the allocation-free scan over words [w0, w1) of chunk ch: the
// work list and pass counters live in the static scratch array, records go to
// d_hits (cap records; the hit count, cleared by the caller, runs on past
// cap). The dense part runs once (dense = true); the sparse part runs again on
// halves of the range while the static work list overflows (its resolve
// kernel then does nothing).
void static_pass(ifa_ctx *c, const DevChunk &ch, uint32_t w0, uint32_t w1, bool dense,
                 ifa_hit *d_hits, uint64_t cap)
{
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(c->scratch);
    ScanArgs a = chunk_args(c, ch);
    a.w_begin = w0;
    a.w_end = w1;
    a.work = reinterpret_cast<WorkItem *>(c->scratch + kScratchCounterBytes);
    a.work_count = reinterpret_cast<unsigned int *>(ctr + 1);
    a.skip_count = a.work_count + 1;
    a.work_cap = kScratchWorkItems;
    a.hits = reinterpret_cast<uint4 *>(d_hits);
    a.hit_count = ctr;
    a.hit_cap = cap;
    PassEvents none;
    enqueue_pass(c, a, false, dense, none);
    if (c->n_sparse == 0 || c->indexed) return;
    hip_check(hipMemcpyAsync(c->h_ctr.p, ctr, 2 * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, c->comp_s),
              "copy pass counters");
    hip_check(hipStreamSynchronize(c->comp_s), "sync");
    const uint32_t items = reinterpret_cast<const unsigned int *>(c->h_ctr.p + 1)[0];
    if (items <= kScratchWorkItems) return;
    // one filter wave's items always fit (checked by the caller)
    if (w1 - w0 <= 32u) fail(IFA_E_DEVICE, "static work list overflow");
    const uint32_t mid = w0 + (w1 - w0) / 2;
    static_pass(c, ch, w0, mid, false, d_hits, cap);
    static_pass(c, ch, mid, w1, false, d_hits, cap);
}

}  // namespace

extern "C" {

void ifa_config_default(ifa_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->abi_version = IFA_ABI_VERSION;
    cfg->device = 0;
    cfg->chunk_bases = 1ull << 30;
    cfg->hit_capacity = 0;
    cfg->strands = IFA_STRAND_BOTH;
    cfg->n_policy = IFA_N_SEPARATE;
    cfg->sink = IFA_SINK_RECORDS;
    cfg->host_threads = 0;
    cfg->flags = IFA_FLAG_GRAPHS;
}

ifa_status ifa_create(const ifa_config *cfg_in, ifa_ctx **out)
{
    if (!out) return IFA_E_INVALID;
    *out = nullptr;
    ifa_config cfg;
    if (cfg_in) cfg = *cfg_in; else ifa_config_default(&cfg);
    if (cfg.abi_version != IFA_ABI_VERSION || cfg.chunk_bases < 4096 ||
        cfg.chunk_bases > (1ull << 31) || (cfg.chunk_bases & 31) || cfg.strands < 1 ||
        cfg.strands > 3 || cfg.n_policy > 1 || cfg.sink > 1 || (cfg.flags & ~(IFA_FLAG_GRAPHS | IFA_FLAG_OVERHANG | IFA_FLAG_INDEXED |
                       IFA_FLAG_AUTO_MODE)) != 0 ||
        ((cfg.flags & (IFA_FLAG_INDEXED | IFA_FLAG_AUTO_MODE)) && (cfg.flags & IFA_FLAG_OVERHANG)))
        return IFA_E_INVALID;
    ifa_ctx *c = new (std::nothrow) ifa_ctx();
    if (!c) return IFA_E_NOMEM;
    c->cfg = cfg;
    ifa_status st = guarded(nullptr, [&]() {
        int ndev = 0;
        hip_check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
        if (cfg.device < 0 || cfg.device >= ndev) fail(IFA_E_INVALID, "no such device");
        use_device(c);
        unsigned hw = std::thread::hardware_concurrency();
        c->threads = cfg.host_threads ? cfg.host_threads : (hw ? hw : 1);
        c->threads = std::min(c->threads, 64u);
        c->plane_words = words_with_pad(cfg.chunk_bases);
        hip_check(hipStreamCreateWithFlags(&c->copy_s, hipStreamNonBlocking), "stream");
        hip_check(hipStreamCreateWithFlags(&c->comp_s, hipStreamNonBlocking), "stream");
        hip_check(hipStreamCreateWithFlags(&c->dense_s, hipStreamNonBlocking), "stream");
        hip_check(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "event");
        hip_check(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming), "event");
        for (int i = 0; i < 2; i++) {
            c->stage[i].planes.alloc(3 * c->plane_words, "pinned staging");
            hip_check(hipEventCreateWithFlags(&c->stage[i].copied, hipEventDisableTiming),
                      "event");
            c->slot[i].stride = c->plane_words;
            c->slot[i].planes.alloc(4 * c->plane_words, "device chunk");
            c->slot[i].pieces.alloc(1024, "device piece table");
            hip_check(hipEventCreateWithFlags(&c->slot[i].free_ev, hipEventDisableTiming),
                      "event");
        }
        uint64_t cap = cfg.hit_capacity;
        if (cap == 0) {
            // 1/32 of the free device memory over the two record buffers,
            // within [2^20, 2^26] records each
            size_t free_b = 0, total_b = 0;
            hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            cap = free_b / 32 / (2 * sizeof(ifa_hit));
            cap = std::min<uint64_t>(std::max<uint64_t>(cap, 1ull << 20), 1ull << 26);
        }
        c->hit_cap = cap;
        if (cfg.sink == IFA_SINK_RECORDS) {
            for (int i = 0; i < 2; i++) {
                c->d_hits[i].alloc(cap, "device hit buffer");
                c->buf_cap[i] = cap;
            }
        }
        const uint32_t wcap = cfg.work_capacity ? cfg.work_capacity : (1u << 22);
        for (int i = 0; i < 2; i++) {
            c->work[i].alloc(wcap, "work list");
            c->work_cap[i] = wcap;
        }
        hipError_t se = hipSuccess;
        c->scratch = static_cast<uint8_t *>(scratch_address(cfg.device, &se));
        hip_check(se, "static scratch address");
        c->d_ctr.alloc(4, "pass counters");
        c->h_ctr.alloc(4, "pinned pass counters");
        hip_check(hipMemset(c->d_ctr.p, 0, 4 * sizeof(unsigned long long)), "memset");
        for (int i = 0; i < 4; i++) c->h_ctr.p[i] = 0;
    });
    if (st != IFA_OK) {
        ifa_destroy(c);
        return st;
    }
    *out = c;
    return IFA_OK;
}

void ifa_destroy(ifa_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    if (c->comp_s) (void)hipStreamSynchronize(c->comp_s);
    if (c->copy_s) (void)hipStreamSynchronize(c->copy_s);
    if (c->dense_s) (void)hipStreamSynchronize(c->dense_s);
    for (auto &pr : c->h2d_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (auto &j : c->jobs) {
        if (j.k0) (void)hipEventDestroy(j.k0);
        if (j.k1) (void)hipEventDestroy(j.k1);
        if (j.kf) (void)hipEventDestroy(j.kf);
        if (j.ke) (void)hipEventDestroy(j.ke);
        if (j.kd) (void)hipEventDestroy(j.kd);
        if (j.kx) (void)hipEventDestroy(j.kx);
        if (j.done) (void)hipEventDestroy(j.done);
    }
    for (int t = 0; t < 2; t++) {
        if (c->qstaged[t]) (void)hipEventDestroy(c->qstaged[t]);
        for (int f = 0; f < 2; f++)
            if (c->mqstaged[t][f]) (void)hipEventDestroy(c->mqstaged[t][f]);
    }
    for (int i = 0; i < 2; i++) {
        if (c->stage[i].copied) (void)hipEventDestroy(c->stage[i].copied);
        if (c->slot[i].free_ev) (void)hipEventDestroy(c->slot[i].free_ev);
    }
    for (auto &r : c->resident)
        if (r->free_ev) (void)hipEventDestroy(r->free_ev);
    c->resident.clear();
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->copy_s) (void)hipStreamDestroy(c->copy_s);
    if (c->comp_s) (void)hipStreamDestroy(c->comp_s);
    if (c->dense_s) (void)hipStreamDestroy(c->dense_s);
    delete c;
}

const char *ifa_last_error(const ifa_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

ifa_status ifa_load_queries(ifa_ctx *c, uint32_t n, const uint8_t *const *seq,
                            const uint32_t *len, const int32_t *max_subs, const int32_t *max_n)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!nothing_pending(c)) fail(IFA_E_STATE, "scans or hits pending; collect hits first");
        validate_queries(n, seq, len, max_subs, max_n);
        use_device(c);
        const bool indexed = (c->cfg.flags & IFA_FLAG_INDEXED) ||
                             ((c->cfg.flags & IFA_FLAG_AUTO_MODE) && n >= c->seedp.auto_queries);
        if (indexed) {
            if (2ull * n >= (1ull << 24)) fail(IFA_E_INVALID, "indexed mode takes < 2^23 queries");
            for (uint32_t j = 0; j < n; j++)
                if (len[j] <= c->seedp.mask)
                    fail(IFA_E_INVALID, "query " + std::to_string(j) +
                                            " is not longer than the seed mask");
        }
        std::vector<QSDesc> qs;
        std::vector<uint32_t> words;
        uint32_t lmax = 0;
        pack_query_strands(c->cfg.strands, n, seq, len, max_subs, max_n, 0, qs, words, lmax,
                           c->threads);
        c->indexed = indexed;
        install_queries(c, std::move(qs), std::move(words), n, lmax);
        if (indexed) install_seeds(c, n, len, max_subs, seq, max_n);
    });
}

ifa_status ifa_scan_chunk(ifa_ctx *c, uint32_t n_contigs, const uint8_t *const *seq,
                          const uint64_t *len, uint32_t *first_ordinal)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        if (n_contigs > 0 && (!seq || !len)) fail(IFA_E_INVALID, "NULL argument");
        for (uint32_t i = 0; i < n_contigs; i++) {
            if (len[i] >= (1ull << 31)) fail(IFA_E_INVALID, "contig longer than 2^31 - 1");
            if (len[i] > 0 && !seq[i]) fail(IFA_E_INVALID, "NULL contig pointer");
        }
        use_device(c);
        if (first_ordinal) *first_ordinal = c->next_ordinal;
        append_contigs(c, n_contigs, seq, len, [&]() { flush_stream(c); });
        // caller memory must not be read after return
        pack_pending(c, c->stage[c->cur]);
    });
}

ifa_status ifa_scan_packed(ifa_ctx *c, const ifa_packed_chunk *pk, uint32_t *first_ordinal)
{
    if (!c || !pk) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        const uint64_t n = pk->n_bases;
        if (n > c->cfg.chunk_bases) fail(IFA_E_INVALID, "packed chunk larger than chunk_bases");
        if (n > 0 && (!pk->hi || !pk->lo)) fail(IFA_E_INVALID, "NULL plane");
        if (pk->n_contigs > 0 && !pk->contig_len) fail(IFA_E_INVALID, "NULL contig table");
        if (pk->n_runs > 0 && (!pk->run_start || !pk->run_len)) fail(IFA_E_INVALID, "NULL N runs");
        uint64_t sum = 0;
        for (uint32_t i = 0; i < pk->n_contigs; i++) {
            if (pk->contig_len[i] >= (1ull << 31)) fail(IFA_E_INVALID, "contig longer than 2^31 - 1");
            sum += pk->contig_len[i];
        }
        if (sum != n) fail(IFA_E_INVALID, "contig lengths do not add up to n_bases");
        for (uint32_t i = 0; i < pk->n_runs; i++) {
            const uint64_t a = pk->run_start[i], len = pk->run_len[i];
            if (len == 0 || a + len > n || (i > 0 && a < pk->run_start[i - 1] + pk->run_len[i - 1]))
                fail(IFA_E_INVALID, "N runs must be non-empty, ascending, disjoint and in the chunk");
        }
        use_device(c);
        if (first_ordinal) *first_ordinal = c->next_ordinal;
        // what was streamed before goes first (ordinals stay in stream order)
        flush_stream(c);
        Staging &s = c->stage[c->cur];
        // pieces: whole contigs back to back; empty contigs take an ordinal only
        uint64_t at = 0;
        for (uint32_t i = 0; i < pk->n_contigs; i++) {
            const uint32_t ordinal = c->next_ordinal++;
            const uint64_t len = pk->contig_len[i];
            if (len == 0) continue;
            Piece p{};
            p.start = at;
            p.len = len;
            p.contig_off = 0;
            p.contig = ordinal;
            p.flags = kPieceContigStart | kPieceContigEnd;
            s.pieces.push_back(p);
            at += len;
        }
        if (n == 0) {
            reset_staging(s);
            return;
        }
        // the planes into pinned staging (the caller may reuse its buffers on
        // return), bits past the last base cleared
        const uint64_t used = (n + 31) >> 5, span = 1ull << 18;
        uint32_t *H = plane(c, s, 0), *Lo = plane(c, s, 1);
        parallel_for(c->threads, (size_t)((used + span - 1) / span), [&](size_t i) {
            const uint64_t w0 = i * span, w1 = std::min<uint64_t>(used, w0 + span);
            std::memcpy(H + w0, pk->hi + w0, (w1 - w0) * sizeof(uint32_t));
            std::memcpy(Lo + w0, pk->lo + w0, (w1 - w0) * sizeof(uint32_t));
        });
        if (n & 31) {
            const uint32_t keep = (1u << (n & 31)) - 1u;
            H[used - 1] &= keep;
            Lo[used - 1] &= keep;
        }
        // N words from the runs (and the chunk tail), then the sparse list
        std::vector<std::pair<uint32_t, uint32_t>> nword;
        auto add = [&](uint64_t w, uint32_t bits) {
            if (!nword.empty() && nword.back().first == (uint32_t)w) nword.back().second |= bits;
            else nword.emplace_back((uint32_t)w, bits);
        };
        for (uint32_t i = 0; i < pk->n_runs; i++) {
            const uint64_t a = pk->run_start[i], b = a + pk->run_len[i];
            for (uint64_t w = a >> 5; w <= (b - 1) >> 5; w++) {
                const uint64_t lo = std::max(a, w << 5), hi = std::min(b, (w + 1) << 5);
                add(w, (uint32_t)(((hi - lo) == 32 ? 0xffffffffull : ((1ull << (hi - lo)) - 1))
                                  << (lo & 31)));
            }
        }
        if (n & 31) add(n >> 5, ~((1u << (n & 31)) - 1u));
        s.len = n;
        s.own_from = 0;
        s.packed_to = n;
        s.n_list = merge_sparse(nword, piece_end_words(s.pieces, n), s.list);
        submit_staging(c);
    });
}

ifa_status ifa_collect_hits(ifa_ctx *c, ifa_hit *out, uint64_t cap, uint64_t *n_written,
                            uint64_t *n_remaining)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (cap > 0 && !out) fail(IFA_E_INVALID, "NULL output");
        use_device(c);
        flush_stream(c);
        retire_all(c);
        if (!c->hits_sorted) {
            std::sort(c->hits.begin() + (ptrdiff_t)c->drain_pos, c->hits.end(),
                      [](const ifa_hit &a, const ifa_hit &b) {
                          if (a.contig != b.contig) return a.contig < b.contig;
                          if (a.pos != b.pos) return a.pos < b.pos;
                          if (a.strand != b.strand) return a.strand < b.strand;
                          return a.query < b.query;
                      });
            c->hits_sorted = true;
        }
        uint64_t avail = c->hits.size() - c->drain_pos;
        uint64_t k = std::min(avail, cap);
        if (k) std::memcpy(out, c->hits.data() + c->drain_pos, k * sizeof(ifa_hit));
        c->drain_pos += k;
        if (n_written) *n_written = k;
        if (n_remaining) *n_remaining = avail - k;
        if (c->drain_pos >= c->hits.size()) {
            c->hits.clear();
            c->hits.shrink_to_fit();
            c->drain_pos = 0;
        }
    });
}

ifa_status ifa_query_stats(ifa_ctx *c, uint64_t *count, uint64_t *digest)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (c->cfg.sink != IFA_SINK_COUNT_DIGEST) fail(IFA_E_STATE, "sink is not count+digest");
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        use_device(c);
        flush_stream(c);
        retire_all(c);
        hip_check(hipStreamSynchronize(c->comp_s), "sync");
        // per-query accumulators are striped over kStripes slots; sum them
        const size_t n = (size_t)c->n_queries * kStripes;
        std::vector<uint64_t> buf(n ? n : 1);
        if (count) {
            hip_check(hipMemcpyAsync(buf.data(), c->d_qcount.p, n * sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, c->comp_s),
                      "copy counts");
            hip_check(hipStreamSynchronize(c->comp_s), "sync count copy");
            for (uint32_t q = 0; q < c->n_queries; q++) {
                uint64_t acc = 0;
                for (uint32_t k = 0; k < kStripes; k++) acc += buf[(size_t)q * kStripes + k];
                count[q] = acc;
            }
        }
        if (digest) {
            hip_check(hipMemcpyAsync(buf.data(), c->d_qdigest.p, n * sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, c->comp_s),
                      "copy digests");
            hip_check(hipStreamSynchronize(c->comp_s), "sync digest copy");
            for (uint32_t q = 0; q < c->n_queries; q++) {
                uint64_t acc = 0;
                for (uint32_t k = 0; k < kStripes; k++) acc += buf[(size_t)q * kStripes + k];
                digest[q] = acc;
            }
        }
    });
}

ifa_status ifa_ref_load(ifa_ctx *c, uint32_t n_contigs, const uint8_t *const *seq,
                        const uint64_t *len, uint32_t *first_ordinal)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (n_contigs > 0 && (!seq || !len)) fail(IFA_E_INVALID, "NULL argument");
        for (uint32_t i = 0; i < n_contigs; i++) {
            if (len[i] >= (1ull << 31)) fail(IFA_E_INVALID, "contig longer than 2^31 - 1");
            if (len[i] > 0 && !seq[i]) fail(IFA_E_INVALID, "NULL contig pointer");
        }
        if (c->stage[c->cur].len != 0)
            fail(IFA_E_STATE, "a streamed chunk is being filled; collect hits first");
        use_device(c);
        if (first_ordinal) *first_ordinal = c->next_ordinal;
        // Build chunks in the streaming staging buffers; each full chunk goes
        // to a new resident device chunk instead of a stream slot.
        auto to_resident = [&]() {
            Staging &s = c->stage[c->cur];
            if (s.len == 0) return;
            pack_pending(c, s);
            seal(c, s);
            std::unique_ptr<DevChunk> d(new DevChunk());
            d->resident = true;
            d->stride = words_with_pad(s.len);
            d->planes.alloc(4 * d->stride, "resident chunk");
            d->pieces.alloc(std::max<size_t>(s.pieces.size(), 1), "resident piece table");
            hip_check(hipEventCreateWithFlags(&d->free_ev, hipEventDisableTiming), "event");
            upload(c, s, *d, c->copy_s);
            hip_check(hipStreamSynchronize(c->copy_s), "sync");
            c->resident_bases += s.len - s.own_from;
            c->resident.push_back(std::move(d));
            reset_staging(s);
        };
        append_contigs(c, n_contigs, seq, len, to_resident);
        to_resident();
        collect_h2d_times(c);
    });
}

ifa_status ifa_scan_resident(ifa_ctx *c)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        if (c->resident.empty()) fail(IFA_E_STATE, "no resident reference");
        use_device(c);
        flush_stream(c);
        for (auto &d : c->resident) {
            c->st.bases += d->len - d->own_from;
            submit_job(c, d.get());
        }
    });
}

ifa_status ifa_scan_resident_into(ifa_ctx *c, ifa_hit *d_hits, uint64_t cap, uint64_t *n_hits)
{
    if (!c || !n_hits) return IFA_E_INVALID;
    return guarded(c, [&]() {
        *n_hits = 0;
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        if (c->resident.empty()) fail(IFA_E_STATE, "no resident reference");
        if (!nothing_pending(c)) fail(IFA_E_STATE, "scans or hits pending; collect hits first");
        if (c->cfg.sink == IFA_SINK_RECORDS && cap > 0 && !d_hits)
            fail(IFA_E_INVALID, "NULL hit buffer");
        uint32_t wpl, qu, wg, enc;
        variant_shape(c->variant, &wpl, &qu, &wg, &enc);
        if (enc >= 1 && c->n_sparse > 0 && !c->indexed && !c->mq_ready[enc == 1 ? 0 : 1])
            fail(IFA_E_STATE, "the variant's filter operands are not built: choose the variant "
                              "before loading the queries");
        // a single filter wave lists at most 32 / list_per items per batch of
        // 32 strands (waves holding an N); the static list must hold one
        // wave's items
        const uint64_t per = list_per(c->n_sparse);
        if ((32u + per - 1u) / per * ((c->n_sparse + 31) / 32) > kScratchWorkItems)
            fail(IFA_E_INVALID, "too many filtered query strands for the static scratch (at most " +
                                    std::to_string(8ull * kScratchWorkItems) + ")");
        use_device(c);
        unsigned long long *ctr = reinterpret_cast<unsigned long long *>(c->scratch);
        // the hit count runs over every chunk: records append to d_hits
        hip_check(launch_clear_u64(ctr, 2, c->comp_s), "clear pass counters");
        for (auto &d : c->resident) {
            static_pass(c, *d, 0, (uint32_t)((d->len + 31) >> 5), true, d_hits, cap);
            c->st.bases += d->len - d->own_from;
            c->st.chunks++;
        }
        hip_check(hipMemcpyAsync(c->h_ctr.p, ctr, sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, c->comp_s),
                  "copy hit count");
        hip_check(hipStreamSynchronize(c->comp_s), "sync");
        const uint64_t n = c->cfg.sink == IFA_SINK_RECORDS ? c->h_ctr.p[0] : 0;
        *n_hits = n;
        if (n > cap)
            fail(IFA_E_NOMEM, "hit buffer holds " + std::to_string(cap) + " records, " +
                                  std::to_string(n) + " needed");
    });
}

ifa_status ifa_ref_release(ifa_ctx *c)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        use_device(c);
        for (auto &j : c->jobs)
            if (j.active) fail(IFA_E_STATE, "scans pending; collect hits first");
        hip_check(hipStreamSynchronize(c->comp_s), "sync");
        for (auto &r : c->resident)
            if (r->free_ev) (void)hipEventDestroy(r->free_ev);
        c->resident.clear();
        c->resident_bases = 0;
    });
}

ifa_status ifa_ref_info(const ifa_ctx *c, uint64_t *bases, uint32_t *chunks)
{
    if (!c) return IFA_E_INVALID;
    if (bases) *bases = c->resident_bases;
    if (chunks) *chunks = (uint32_t)c->resident.size();
    return IFA_OK;
}

ifa_status ifa_get_stats(ifa_ctx *c, ifa_stats *out)
{
    if (!c || !out) return IFA_E_INVALID;
    return guarded(c, [&]() {
        use_device(c);
        retire_all(c);
        *out = c->st;
    });
}

ifa_status ifa_set_graphs(ifa_ctx *c, int enable)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        use_device(c);
        retire_all(c);
        if (enable) c->cfg.flags |= IFA_FLAG_GRAPHS;
        else c->cfg.flags &= ~IFA_FLAG_GRAPHS;
    });
}

ifa_status ifa_set_overlap(ifa_ctx *c, int enable)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        use_device(c);
        retire_all(c);
        c->overlap = enable != 0;
    });
}

uint32_t ifa_variant_count(void) { return ifa::variant_count(); }

ifa_status ifa_variant_info(uint32_t v, uint32_t *windows_per_lane, uint32_t *queries_per_iter,
                            uint32_t *workgroup, uint32_t *encoding)
{
    if (v >= ifa::variant_count()) return IFA_E_INVALID;
    uint32_t a, b, g, e;
    ifa::variant_shape(v, &a, &b, &g, &e);
    if (windows_per_lane) *windows_per_lane = a;
    if (queries_per_iter) *queries_per_iter = b;
    if (workgroup) *workgroup = g;
    if (encoding) *encoding = e;
    return IFA_OK;
}

ifa_status ifa_set_variant(ifa_ctx *c, uint32_t v)
{
    if (!c) return IFA_E_INVALID;
    if (v >= ifa::variant_count()) {
        c->err = "no such kernel variant";
        return IFA_E_INVALID;
    }
    c->variant = v;
    return IFA_OK;
}

ifa_status ifa_get_variant(const ifa_ctx *c, uint32_t *v)
{
    if (!c || !v) return IFA_E_INVALID;
    *v = c->variant;
    return IFA_OK;
}

ifa_status ifa_autotune(ifa_ctx *c, uint64_t calib_bases, uint32_t reps, const char *cache_path,
                        uint32_t *chosen, double *ms_per_variant)
{
    if (!c) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!c->have_queries) fail(IFA_E_STATE, "no queries loaded");
        if (!nothing_pending(c)) fail(IFA_E_STATE, "scans or hits pending; collect hits first");
        use_device(c);
        if (calib_bases == 0) calib_bases = 64ull << 20;
        calib_bases = std::max<uint64_t>(4096, std::min<uint64_t>(calib_bases, c->cfg.chunk_bases));
        calib_bases &= ~31ull;
        if (reps == 0) reps = 3;
        const std::string key = tune_key(c);
        const uint32_t nv = ifa::variant_count();
        if (cache_path) {
            uint32_t v;
            if (cache_lookup(cache_path, key, &v) && v < nv) {
                c->variant = v;
                if (chosen) *chosen = v;
                if (ms_per_variant)
                    for (uint32_t i = 0; i < nv; i++) ms_per_variant[i] = -1.0;
                return;
            }
        }
        // calibration chunk: uniform random bases, one contig piece, no N
        DevChunk ch;
        ch.stride = words_with_pad(calib_bases);
        ch.planes.alloc(4 * ch.stride, "calibration chunk");
        ch.pieces.alloc(1, "calibration piece");
        const uint64_t used = calib_bases >> 5;
        std::vector<uint32_t> host(2 * used, 0u);
        uint64_t z = 0x243F6A8885A308D3ull;
        for (uint64_t w = 0; w < used; w++) {
            z += 0x9E3779B97F4A7C15ull;
            uint64_t r = z;
            r = (r ^ (r >> 30)) * 0xBF58476D1CE4E5B9ull;
            r = (r ^ (r >> 27)) * 0x94D049BB133111EBull;
            r ^= r >> 31;
            host[w] = (uint32_t)r;
            host[used + w] = (uint32_t)(r >> 32);
        }
        const uint4 end_word{(uint32_t)((calib_bases - 1) >> 5), 0u,
                             1u << ((calib_bases - 1) & 31), 0u};
        upload_planes(host.data(), host.data() + used, used, &end_word, 1, ch, c->comp_s);
        Piece pc{};
        pc.len = calib_bases;
        hip_check(hipMemcpyAsync(ch.pieces.p, &pc, sizeof pc, hipMemcpyHostToDevice, c->comp_s),
                  "upload piece");
        hip_check(hipStreamSynchronize(c->comp_s), "sync calibration upload");
        ch.len = calib_bases;
        ch.n_pieces = 1;
        // hits go to the context's kind of sink in scratch memory (a small
        // record buffer, or scratch per-query counters: the sinks differ in
        // cost when hits are dense) and the work list to a scratch list; the
        // tuner only times (a full scratch list skips the resolve)
        DevBuf<uint4> scratch_hits;
        scratch_hits.alloc(1024, "tuning hit buffer");
        DevBuf<unsigned long long> scratch_cnt;
        scratch_cnt.alloc(2, "tuning counter");
        DevBuf<unsigned long long> scratch_qc, scratch_qd;
        const bool digest = c->cfg.sink == IFA_SINK_COUNT_DIGEST;
        if (digest) {
            const size_t need = (size_t)std::max<uint32_t>(c->n_queries, 1) * kStripes;
            scratch_qc.alloc(need, "tuning query counters");
            scratch_qd.alloc(need, "tuning query digests");
        }
        // the work list holds what a variant's filter lists (it grows and the
        // variant is timed again when it overflows: an overflowing list skips
        // the resolve kernel, which would flatter a weak filter)
        uint32_t work_cap = 1u << 16;
        DevBuf<WorkItem> scratch_work;
        scratch_work.alloc(work_cap, "tuning work list");
        DevBuf<unsigned int> scratch_wc;
        scratch_wc.alloc(2, "tuning work counters");
        hipEvent_t e0, e1;
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
        std::vector<double> ms(nv, 0.0);
        const uint32_t saved = c->variant;
        for (uint32_t v = 0; v < nv; v++) {
            c->variant = v;
            ScanArgs a = make_args(c, ch, 0);
            a.sink = digest ? kSinkCountDigest : kSinkRecords;
            a.hits = scratch_hits.p;
            a.hit_count = scratch_cnt.p;
            a.hit_cap = 1024;
            a.q_count = scratch_qc.p;
            a.q_digest = scratch_qd.p;
            a.work_count = scratch_wc.p;
            a.skip_count = scratch_wc.p + 1;
            // the kernels as a pass runs them: with the overlap on (and both
            // kinds of strand), the dense kernels beside the filter
            auto pass = [&]() {
                hip_check(launch_clear_u32(a.work_count, 2, c->comp_s), "clear");
                const bool side = forks(c, a, true);
                if (side) {
                    hip_check(hipEventRecord(c->fork_ev, c->comp_s), "fork");
                    hip_check(hipStreamWaitEvent(c->dense_s, c->fork_ev, 0), "fork");
                    hip_check(launch_dense(a, c->dense_s), "tuning launch");
                    hip_check(hipEventRecord(c->join_ev, c->dense_s), "join");
                }
                hip_check(launch_filter(a, c->comp_s), "tuning launch");
                hip_check(launch_resolve(a, c->comp_s), "tuning launch");
                if (side)
                    hip_check(hipStreamWaitEvent(c->comp_s, c->join_ev, 0), "join");
                else
                    hip_check(launch_dense(a, c->comp_s), "tuning launch");
            };
            for (;;) {
                a.work = scratch_work.p;
                a.work_cap = work_cap;
                pass();   // warm up, and the list's need
                unsigned int items = 0;
                hip_check(hipMemcpyAsync(&items, scratch_wc.p, sizeof items,
                                         hipMemcpyDeviceToHost, c->comp_s),
                          "copy tuning work count");
                hip_check(hipStreamSynchronize(c->comp_s), "sync tuning pass");
                if (items <= work_cap || work_cap >= (1u << 28)) break;
                work_cap = (uint32_t)std::min<uint64_t>(2ull * items, 1ull << 28);
                scratch_work.alloc(work_cap, "tuning work list");
            }
            std::vector<float> t(reps);
            for (uint32_t r = 0; r < reps; r++) {
                hip_check(hipEventRecord(e0, c->comp_s), "event record");
                pass();
                hip_check(hipEventRecord(e1, c->comp_s), "event record");
                hip_check(hipEventSynchronize(e1), "tuning sync");
                hip_check(hipEventElapsedTime(&t[r], e0, e1), "event time");
            }
            std::sort(t.begin(), t.end());
            ms[v] = t[reps / 2];
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->variant = saved;
        uint32_t best = 0;
        for (uint32_t v = 1; v < nv; v++)
            if (ms[v] < ms[best]) best = v;
        c->variant = best;
        c->tune_ms = ms;
        if (chosen) *chosen = best;
        if (ms_per_variant)
            for (uint32_t i = 0; i < nv; i++) ms_per_variant[i] = ms[i];
        if (cache_path) cache_store(cache_path, key, best, ms[best]);
    });
}

ifa_status ifa_query_partition(const ifa_ctx *c, uint32_t *n_strands, uint32_t *n_filtered)
{
    if (!c) return IFA_E_INVALID;
    if (n_strands) *n_strands = (uint32_t)c->h_qs.size();
    if (n_filtered) *n_filtered = c->n_sparse;
    return IFA_OK;
}

ifa_status ifa_device_footprint(const ifa_ctx *c, uint64_t *bytes)
{
    if (!c || !bytes) return IFA_E_INVALID;
    uint64_t b = 0;
    for (int i = 0; i < 2; i++) {
        b += c->slot[i].planes.n * sizeof(uint32_t) + c->slot[i].pieces.n * sizeof(Piece);
        b += c->d_hits[i].n * sizeof(uint4) + c->work[i].n * sizeof(WorkItem);
    }
    b += c->d_ctr.n * sizeof(unsigned long long);
    for (int t = 0; t < 2; t++)
        b += c->d_qarena[t].n + c->d_mqarena[t][0].n + c->d_mqarena[t][1].n;
    b += (c->d_qcount.n + c->d_qdigest.n) * sizeof(unsigned long long);
    b += c->d_seed_info.n * sizeof(SeedInfo) + c->d_seed_tab.n * sizeof(SeedTable);
    for (size_t i = 0; i < kMaxSeedCfg; i++)
        b += (c->d_seed_dir[i].n + c->d_seed_ent[i].n + c->d_seed_bm[i].n) * sizeof(uint32_t);
    for (const auto &r : c->resident)
        b += r->planes.n * sizeof(uint32_t) + r->pieces.n * sizeof(Piece);
    *bytes = b;
    return IFA_OK;
}

void ifa_index_params_default(ifa_index_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    const uint32_t ks[] = {8, 9, 10, 12, 14};
    p->n_k = 5;
    for (uint32_t i = 0; i < 5; i++) p->k[i] = ks[i];
    p->mask = 0;
    p->step = 1;
    p->prob_ppm = 999000;
    p->iters = 200000;
    p->seed = 1;
    p->auto_queries = kAutoQueries;
}

ifa_status ifa_query_mode(const ifa_ctx *c, uint32_t *indexed)
{
    if (!c || !indexed) return IFA_E_INVALID;
    if (!c->have_queries) return IFA_E_STATE;
    *indexed = c->indexed ? 1u : 0u;
    return IFA_OK;
}

ifa_status ifa_set_index_params(ifa_ctx *c, const ifa_index_params *p)
{
    if (!c || !p) return IFA_E_INVALID;
    return guarded(c, [&]() {
        if (!(c->cfg.flags & (IFA_FLAG_INDEXED | IFA_FLAG_AUTO_MODE)))
            fail(IFA_E_INVALID, "not an indexed or auto-mode context");
        if (p->n_k < 1 || p->n_k > IFA_MAX_SEED_KS || p->step < 1 || p->prob_ppm > 1000000u ||
            p->iters < 1 || p->iters > (1ull << 31))
            fail(IFA_E_INVALID, "bad index parameters");
        for (uint32_t i = 0; i < p->n_k; i++)
            if (p->k[i] <= p->mask || p->k[i] > 16) fail(IFA_E_INVALID, "seed length out of range");
        SeedParams q;
        q.n_k = p->n_k;
        for (uint32_t i = 0; i < p->n_k; i++) q.k[i] = p->k[i];
        q.mask = p->mask;
        q.step = p->step;
        q.ppm = p->prob_ppm;
        q.iters = p->iters;
        q.seed = p->seed;
        q.auto_queries = p->auto_queries;
        const bool same = q.mask == c->seedp.mask && q.step == c->seedp.step &&
                          q.ppm == c->seedp.ppm && q.iters == c->seedp.iters &&
                          q.seed == c->seedp.seed;
        if (!same) c->mh_cache.clear();
        c->seedp = q;
    });
}

ifa_status ifa_query_seeds(const ifa_ctx *c, uint32_t *k, uint32_t *thr)
{
    if (!c) return IFA_E_INVALID;
    if (!c->indexed || !c->have_queries) return IFA_E_STATE;
    if (k)
        for (uint32_t j = 0; j < c->n_queries; j++) k[j] = c->seeds.qk[j];
    if (thr)
        for (size_t j = 0; j < 2 * (size_t)c->n_queries; j++) thr[j] = c->seeds.qthr[j];
    return IFA_OK;
}

ifa_status ifa_reset_stats(ifa_ctx *c)
{
    if (!c) return IFA_E_INVALID;
    std::memset(&c->st, 0, sizeof c->st);
    return IFA_OK;
}

}  // extern "C"

// ===========================================================================
// Serving loop: continuous batching over a device-resident reference
// ===========================================================================
//
// Requests (query sets with their own thresholds) arrive at any time. A step
// scans one resident chunk, the one under a rotating cursor, with the union
// of the query strands of every admitted request, so the work of different
// requests overlaps in the same kernels. A request admitted at step s sees
// the chunks s, s+1, ... (mod the chunk count) and completes after one full
// revolution; its hits are then sorted into reference order.
//
// Steps are pipelined: step t submits the scan of its chunk and only then
// waits for the scan of step t - 1 and routes its hits to their requests, so
// the host's routing and the next table build overlap the device's work. The
// union query table is rebuilt only when the active set changes; the context
// alternates between two sets of query tables, so a new table is uploaded
// while the previous step's scan still reads the old one.
//
// Admission keeps the active query count under a cap (bounding step time)
// and the hits one step can produce under a record budget: each request
// reserves, per chunk, the binomial expectation of its hits on iid bases
// plus six standard deviations and a floor of 1,024 records. The budget is
// given, or (0) a quarter of the device memory free when the server is
// created, spread over the context's two hit buffers. The hit buffers grow to
// the admitted reservation. A request alone on the server is always admitted
// (a chunk whose hits overflow the buffer is re-scanned in halves).

namespace {

struct SrvRequest {
    uint64_t id = 0;
    uint32_t n_queries = 0;
    std::vector<QSDesc> qs;           // qid = query index within the request
    std::vector<uint32_t> words;
    uint32_t lmax = 0;
    uint32_t chunks_left = 0;         // chunk scans still to submit
    uint32_t routed_left = 0;         // chunk scans whose hits are not routed yet
    double reserve = 0.0;             // hit records reserved per chunk
    std::vector<ifa_hit> hits;
};

// The installed union table: its requests in table order and the first
// table query index of each.
struct SrvTable {
    std::vector<SrvRequest *> reqs;
    std::vector<uint32_t> base;
};

}  // namespace

struct ifa_server {
    ifa_ctx *ctx = nullptr;
    uint32_t max_active_queries = 0;
    uint64_t hit_budget = 0;          // records per step (both hit buffers hold it)
    std::deque<std::unique_ptr<SrvRequest>> pending;
    std::vector<std::unique_ptr<SrvRequest>> active;     // admitted, chunks left to scan
    std::vector<std::unique_ptr<SrvRequest>> finishing;  // scanned, hits not all routed
    std::deque<std::unique_ptr<SrvRequest>> done;
    uint32_t active_queries = 0;
    double active_reserve = 0.0;
    bool table_dirty = true;          // the active set changed since the table was built
    std::shared_ptr<SrvTable> table;  // installed union table
    std::deque<std::shared_ptr<SrvTable>> inflight;   // tables of submitted, unrouted scans
    uint32_t cursor = 0;
    uint64_t next_id = 1;
    uint64_t steps = 0;
    uint64_t completed = 0;
    double step_ms = 0.0;
};

namespace {

// Hit records a request reserves per chunk of `bases` reference bases: the
// expected hits on iid uniform bases (each base matches with probability
// 1/4), plus 6 standard deviations and a floor.
double hit_reserve(const SrvRequest &r, uint64_t bases)
{
    double e = 0.0, v = 0.0;
    for (const QSDesc &d : r.qs) {
        const double p = binom_cdf(d.len, 0.75, d.k);
        e += (double)bases * p;
        v += (double)bases * p * (1.0 - p);
    }
    return e + 6.0 * std::sqrt(v) + 1024.0;
}

uint64_t largest_chunk(const ifa_ctx *c)
{
    uint64_t m = 0;
    for (const auto &d : c->resident) m = std::max<uint64_t>(m, d->len);
    return m;
}

void server_admit(ifa_server *S)
{
    while (!S->pending.empty()) {
        SrvRequest &r = *S->pending.front();
        const bool alone = S->active.empty();
        if (!alone && (S->active_queries + r.n_queries > S->max_active_queries ||
                       S->active_reserve + r.reserve > (double)S->hit_budget))
            break;
        r.chunks_left = (uint32_t)S->ctx->resident.size();
        r.routed_left = r.chunks_left;
        S->active_queries += r.n_queries;
        S->active_reserve += r.reserve;
        S->active.push_back(std::move(S->pending.front()));
        S->pending.pop_front();
        S->table_dirty = true;
    }
}

// Install one query table for every active request: qid = the request's
// table base + its local index.
void server_install(ifa_server *S)
{
    ifa_ctx *c = S->ctx;
    std::shared_ptr<SrvTable> t = std::make_shared<SrvTable>();
    std::vector<QSDesc> qs;
    std::vector<uint32_t> words;
    uint32_t lmax = 0, nq = 0;
    for (auto &rp : S->active) {
        const SrvRequest &r = *rp;
        const uint32_t wb = (uint32_t)words.size();
        t->reqs.push_back(rp.get());
        t->base.push_back(nq);
        for (QSDesc d : r.qs) {
            d.qid += nq;
            d.woff += wb;
            qs.push_back(d);
        }
        words.insert(words.end(), r.words.begin(), r.words.end());
        nq += r.n_queries;
        lmax = std::max(lmax, r.lmax);
    }
    c->indexed = false;   // serving runs brute-force passes
    install_queries(c, std::move(qs), std::move(words), nq, lmax);
    S->table = t;
    S->table_dirty = false;
}

// Wait for the oldest submitted scan and route its hits to their requests;
// requests whose last scan this was are complete.
void server_route_oldest(ifa_server *S)
{
    ifa_ctx *c = S->ctx;
    const std::shared_ptr<SrvTable> t = S->inflight.front();
    S->inflight.pop_front();
    const uint64_t seq = c->job_seq - 1 - S->inflight.size();   // that scan's job
    retire(c, c->jobs[seq % 2]);
    for (const ifa_hit &h : c->hits) {
        const size_t i = (size_t)(std::upper_bound(t->base.begin(), t->base.end(), h.query) -
                                  t->base.begin()) - 1;
        ifa_hit local = h;
        local.query = h.query - t->base[i];
        t->reqs[i]->hits.push_back(local);
    }
    c->hits.clear();
    c->drain_pos = 0;
    c->hits_sorted = true;
    for (SrvRequest *r : t->reqs) r->routed_left--;
    std::vector<std::unique_ptr<SrvRequest>> still;
    for (auto &rp : S->finishing) {
        if (rp->routed_left == 0) {
            std::sort(rp->hits.begin(), rp->hits.end(), [](const ifa_hit &a, const ifa_hit &b) {
                if (a.contig != b.contig) return a.contig < b.contig;
                if (a.pos != b.pos) return a.pos < b.pos;
                if (a.strand != b.strand) return a.strand < b.strand;
                return a.query < b.query;
            });
            S->completed++;
            S->done.push_back(std::move(rp));
        } else {
            still.push_back(std::move(rp));
        }
    }
    S->finishing.swap(still);
}

void server_step(ifa_server *S)
{
    ifa_ctx *c = S->ctx;
    server_admit(S);
    if (S->active.empty() && S->inflight.empty()) return;
    const double t0 = now_ms();
    if (!S->active.empty()) {
        if (S->table_dirty) server_install(S);
        // both hit buffers hold the admitted reservation (they only grow;
        // neither is in use by an unretired scan of the other buffer)
        const uint64_t want = (uint64_t)std::min(S->active_reserve, (double)S->hit_budget);
        const int hb = (int)(c->job_seq % 2);
        if (c->buf_cap[hb] < want) {
            c->d_hits[hb].alloc(want, "grow hit buffer");
            c->buf_cap[hb] = want;
        }
        DevChunk *ch = c->resident[S->cursor].get();
        c->st.bases += ch->len - ch->own_from;
        submit_job(c, ch);
        S->inflight.push_back(S->table);
        S->cursor = (S->cursor + 1) % (uint32_t)c->resident.size();
        S->steps++;
        // requests that have had every chunk submitted leave the active set
        std::vector<std::unique_ptr<SrvRequest>> still;
        for (auto &rp : S->active) {
            if (--rp->chunks_left == 0) {
                S->active_queries -= rp->n_queries;
                S->active_reserve -= rp->reserve;
                S->finishing.push_back(std::move(rp));
                S->table_dirty = true;
            } else {
                still.push_back(std::move(rp));
            }
        }
        S->active.swap(still);
        if (S->active.empty()) S->active_reserve = 0.0;
    }
    // route the previous step's scan while this one runs (or, with nothing
    // new submitted, drain the last one)
    while (S->inflight.size() > 1 || (!S->inflight.empty() && S->active.empty()))
        server_route_oldest(S);
    S->step_ms += now_ms() - t0;
}

}  // namespace

extern "C" {

void ifa_server_config_default(ifa_server_config *cfg)
{
    if (!cfg) return;
    cfg->max_active_queries = 4096;
    cfg->reserved = 0;
    cfg->hit_budget = 0;
}

ifa_status ifa_server_create(ifa_ctx *c, const ifa_server_config *cfg_in, ifa_server **out)
{
    if (!c || !out) return IFA_E_INVALID;
    *out = nullptr;
    return guarded(c, [&]() {
        if (c->resident.empty()) fail(IFA_E_STATE, "no resident reference: call ifa_ref_load");
        if (c->cfg.sink != IFA_SINK_RECORDS) fail(IFA_E_STATE, "serving needs the records sink");
        if (c->cfg.flags & IFA_FLAG_INDEXED) fail(IFA_E_STATE, "serving runs brute-force mode");
        if (!nothing_pending(c)) fail(IFA_E_STATE, "scans or hits pending; collect hits first");
        ifa_server_config cfg;
        if (cfg_in) cfg = *cfg_in; else ifa_server_config_default(&cfg);
        if (cfg.max_active_queries == 0 || cfg.reserved != 0)
            fail(IFA_E_INVALID, "bad server config");
        uint64_t budget = cfg.hit_budget;
        if (budget == 0) {
            // a quarter of the free device memory, over the two hit buffers
            use_device(c);
            size_t free_b = 0, total_b = 0;
            hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            budget = std::max<uint64_t>(free_b / 4 / (2 * sizeof(ifa_hit)), 1u << 16);
        }
        ifa_server *S = new ifa_server();
        S->ctx = c;
        S->max_active_queries = cfg.max_active_queries;
        S->hit_budget = budget;
        *out = S;
    });
}

void ifa_server_destroy(ifa_server *S)
{
    if (!S) return;
    if (S->ctx) {
        ifa_ctx *c = S->ctx;
        (void)hipSetDevice(c->cfg.device);
        // scans still in flight are retired and their hits dropped, so the
        // context is left with nothing pending
        (void)guarded(c, [&]() {
            retire_all(c);
            c->hits.clear();
            c->drain_pos = 0;
            c->hits_sorted = true;
        });
        if (c->comp_s) (void)hipStreamSynchronize(c->comp_s);
    }
    delete S;
}

ifa_status ifa_server_submit(ifa_server *S, uint32_t n, const uint8_t *const *seq,
                             const uint32_t *len, const int32_t *max_subs, const int32_t *max_n,
                             uint64_t *request_id)
{
    if (!S) return IFA_E_INVALID;
    ifa_ctx *c = S->ctx;
    return guarded(c, [&]() {
        if (n == 0) fail(IFA_E_INVALID, "empty request");
        validate_queries(n, seq, len, max_subs, max_n);
        std::unique_ptr<SrvRequest> r(new SrvRequest());
        r->id = S->next_id++;
        r->n_queries = n;
        pack_query_strands(c->cfg.strands, n, seq, len, max_subs, max_n, 0, r->qs, r->words,
                           r->lmax, c->threads);
        r->reserve = hit_reserve(*r, largest_chunk(c));
        if (request_id) *request_id = r->id;
        S->pending.push_back(std::move(r));
    });
}

ifa_status ifa_server_step(ifa_server *S, uint32_t *n_active, uint32_t *n_done_waiting)
{
    if (!S) return IFA_E_INVALID;
    ifa_ctx *c = S->ctx;
    return guarded(c, [&]() {
        use_device(c);
        server_step(S);
        if (n_active) *n_active = (uint32_t)S->active.size();
        if (n_done_waiting) *n_done_waiting = (uint32_t)S->done.size();
    });
}

ifa_status ifa_server_poll(ifa_server *S, uint64_t *request_id, uint64_t *n_hits)
{
    if (!S || !request_id) return IFA_E_INVALID;
    if (S->done.empty()) {
        *request_id = 0;
        if (n_hits) *n_hits = 0;
        return IFA_OK;
    }
    *request_id = S->done.front()->id;
    if (n_hits) *n_hits = S->done.front()->hits.size();
    return IFA_OK;
}

ifa_status ifa_server_take(ifa_server *S, uint64_t request_id, ifa_hit *out, uint64_t cap)
{
    if (!S) return IFA_E_INVALID;
    ifa_ctx *c = S->ctx;
    return guarded(c, [&]() {
        if (S->done.empty() || S->done.front()->id != request_id)
            fail(IFA_E_STATE, "request is not the next completed one (call ifa_server_poll)");
        SrvRequest &r = *S->done.front();
        if (cap < r.hits.size()) fail(IFA_E_INVALID, "output array too small");
        if (!r.hits.empty()) {
            if (!out) fail(IFA_E_INVALID, "NULL output");
            std::memcpy(out, r.hits.data(), r.hits.size() * sizeof(ifa_hit));
        }
        S->done.pop_front();
    });
}

ifa_status ifa_server_info(const ifa_server *S, ifa_server_stats *out)
{
    if (!S || !out) return IFA_E_INVALID;
    out->pending = (uint32_t)S->pending.size();
    out->active = (uint32_t)S->active.size();
    out->active_queries = S->active_queries;
    out->done_waiting = (uint32_t)S->done.size();
    out->steps = S->steps;
    out->completed = S->completed;
    out->step_ms = S->step_ms;
    out->cursor = S->cursor;
    out->chunks = (uint32_t)S->ctx->resident.size();
    out->hit_budget = S->hit_budget;
    out->hits_reserved = (uint64_t)S->active_reserve;
    out->in_flight = (uint32_t)S->inflight.size();
    out->finishing = (uint32_t)S->finishing.size();
    return IFA_OK;
}

}  // extern "C"
