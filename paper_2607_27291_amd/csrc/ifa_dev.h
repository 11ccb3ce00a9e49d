// ifa_dev.h -- data layouts shared by the host runtime and the gfx950 kernels.
//
// Reference chunk in device memory: four bit planes of `plane_words` uint32
// words each, stored one after another (hi, lo, nm, em). Base x of the chunk
// is bit (x & 31) of word (x >> 5) in every plane:
//   hi, lo : 2-bit base code A=00 C=01 G=11 T=10 (hi bit, lo bit): bits 2
//            and 1 of the ASCII byte; complementing a base flips hi
//   nm     : 1 where the base is N (any non-ACGT byte)
//   em     : 1 at the last base of every contig piece, so a window is inside
//            one piece iff no em bit falls on its first L-1 positions
// hi/lo bits at N positions are unspecified (readers mask them with nm).
// Words past the chunk end hold hi = lo = 0 and nm = em = all ones, and at
// least IFA_PAD_WORDS such words follow the last data word.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace ifa {

constexpr uint32_t kMaxLen = 256;          // layout bound: queries are at most 255 bases
constexpr uint32_t kCarry = kMaxLen - 1;   // bases repeated at a split
constexpr uint32_t kPadWords = 16;         // > (31 + kMaxLen) / 32 + 1
constexpr uint32_t kMaxQWords = kMaxLen / 32;
// Static scratch of the allocation-free entry point: kScratchCounterBytes of
// pass counters (hit count u64, work count u32, skipped waves u32), then
// kScratchWorkItems work-list items.
constexpr uint32_t kScratchCounterBytes = 256;
constexpr uint32_t kScratchWorkItems = 1u << 20;
constexpr uint64_t kScratchBytes = kScratchCounterBytes + 16ull * kScratchWorkItems;
// count+digest accumulators are striped: query q adds into slot
// q * kStripes + (workgroup % kStripes); the host sums the stripes
constexpr uint32_t kStripes = 64;

enum Sink : uint32_t { kSinkRecords = 0, kSinkCountDigest = 1 };
enum Policy : uint32_t { kNSeparate = 0, kNAsMismatch = 1 };

// One contig piece inside a chunk.
struct Piece {
    uint64_t start;       // chunk-local offset of the first base
    uint64_t len;         // bases
    uint64_t contig_off;  // contig coordinate of the first base
    uint32_t contig;      // global contig ordinal
    uint32_t flags;       // kPieceContigStart | kPieceContigEnd
};
// Piece.flags: the piece holds the contig's first base (contig_off == 0) /
// its last base.
constexpr uint32_t kPieceContigStart = 1u;
constexpr uint32_t kPieceContigEnd = 2u;
static_assert(sizeof(Piece) == 32, "Piece layout");

// One (query, strand) entry, 32 bytes so a wave reads it with a single scalar
// load. Its packed words live at qwords[woff ...]: for word t (bases 32t ..
// 32t+31 of the strand sequence) the three words hi, lo, qn at
// woff + 3t + {0, 1, 2}; bits at or past L are zero. Word 0 is repeated
// inline (qh0, ql0, qn0) for the filter.
struct QSDesc {
    uint32_t qid;         // caller's query index
    uint16_t len;         // L
    uint8_t strand;       // 0 forward, 1 reverse complement
    uint8_t nw;           // ceil(L / 32)
    uint16_t k;           // min(maxSubs, L)
    uint16_t maxn;        // min(maxN, L)
    uint32_t woff;
    uint32_t qh0, ql0, qn0;
    uint32_t thr;         // filter bound on the first min(L, 32) bases (= k);
                          // >= 32: the filter cannot exclude a window
};
static_assert(sizeof(QSDesc) == 32, "QSDesc layout");

// Indexed mode: per query strand, its seed length, the error-free seeds a
// hit needs, and the offsets where a seed starts (sampled every `step` bases,
// no N at an unmasked position): bit i of valid[i / 32].
constexpr uint32_t kMaxSeedCfg = 8;   // distinct seed lengths of one query set
struct SeedInfo {
    uint32_t k;
    uint32_t thr;
    uint32_t pad[2];
    uint32_t valid[kMaxQWords];
};
static_assert(sizeof(SeedInfo) == 48, "SeedInfo layout");

// Indexed mode: one seed table per distinct seed length k of the query set:
// 2^bits buckets, bucket b = (key * 0x9E3779B1) >> (32 - bits) holding the
// entries ent[dir[b] .. dir[b + 1]), entry = (key, strand << 8 | offset).
// key = the seed's hi bits then lo bits, its masked centre squeezed out.
struct SeedTable {
    uint32_t k;
    uint32_t bits;
    const uint32_t *dir;
    const uint2 *ent;
    // presence bitmap of the table's keys: bit seed_bit(key) is set for every
    // key of the table (a key absent from it needs no directory read)
    const uint32_t *bm;
    uint32_t key_bits;    // 2 (k - mask): bits of a key
    uint32_t pad;
};
static_assert(sizeof(SeedTable) == 40, "SeedTable layout");

// Keys of up to kSeedBitmapBits bits index the presence bitmap directly (it
// is exact); longer keys index it by the top kSeedBitmapBits bits of their
// Fibonacci hash (a one-hash Bloom filter). Bitmap bits: 2^min(key_bits, 28).
constexpr uint32_t kSeedBitmapBits = 28;
__host__ __device__ inline uint32_t seed_bitmap_bits(uint32_t key_bits)
{
    return key_bits < kSeedBitmapBits ? key_bits : kSeedBitmapBits;
}
__host__ __device__ inline uint32_t seed_bit(uint32_t key, uint32_t key_bits)
{
    return key_bits <= kSeedBitmapBits ? key : (key * 0x9E3779B1u) >> (32u - kSeedBitmapBits);
}

// Work item of the sparse path: wave `wave` of the filter grid has at least
// one candidate window for the query strands qb + j, j a set bit of `pending`.
struct WorkItem {
    uint32_t wave;
    uint32_t qb;
    uint32_t pending;
    uint32_t pad;
};
static_assert(sizeof(WorkItem) == 16, "WorkItem layout");

// N-block flags of a chunk whose planes hold `total` words (padding
// included): one byte per 32-word block, plus two so that a filter wave may
// read the flags of the three blocks its words can touch.
__host__ __device__ inline uint32_t nflag_blocks(uint32_t total) { return (total + 31u) / 32u + 2u; }

struct ScanArgs {
    const uint32_t *hi, *lo, *nm, *em;
    const uint8_t *nflag;     // per 32-word block: an N bit, or words past the data
    uint64_t chunk_len;       // bases in the chunk
    uint32_t own_from;        // a window is owned only if its last base >= own_from
    uint32_t w_begin, w_end;  // window-start words [w_begin, w_end) to scan
    uint32_t lmax;            // longest L among qs
    const QSDesc *qs;
    uint32_t n_qs;            // query strands; [0, n_sparse) filtered, the rest dense
    uint32_t n_sparse;
    uint32_t policy;
    // strands per work item when a filter wave lists a whole batch for the
    // resolve kernel (a wave holding an N): 1, 2, 4 or 8
    uint32_t list_per;
    const uint32_t *qwords;
    const Piece *pieces;
    uint32_t n_pieces;
    uint32_t sink;
    uint32_t variant;         // kernel variant index (see kVariants)
    // records sink
    uint4 *hits;
    unsigned long long *hit_count;
    unsigned long long hit_cap;
    // sparse-path work list (filled by the filter kernel, read by resolve)
    WorkItem *work;
    unsigned int *work_count;
    unsigned int *skip_count;   // waves the filter handed whole to the resolve kernel
    unsigned int work_cap;
    // matrix-core filter operands for the sparse strands, two strands (x 16
    // shifts) per 32-column tile: mq_b[(3 tile + K step) * 64 + lane] is the
    // lane's fp4 B operand, mq_t[32 tile + column] the match count a window
    // needs to stay a candidate (padding columns: unreachable)
    const uint4 *mq_b;
    const float *mq_t;
    // three-class form: four strands (x 8 shifts) per tile, two K steps per
    // 32-base prefix word, up to two words:
    // mq3_b[((2 tile + word) * 2 + K step) * 64 + lane], mq3_t[32 tile + column],
    // mq3_w[tile] = words the tile filters on; mq3_words = their maximum
    const uint4 *mq3_b;
    const float *mq3_t;
    const uint32_t *mq3_w;
    uint32_t mq3_words;
    uint32_t mq3_two_batches;   // batches [0, this) hold every two-word tile
    // matrix-core filters: batch of 32 strands of grid row 0 (the grid's y
    // dimension holds at most 65535 batches per launch)
    uint32_t batch0;
    // dense strands [dm_first, n_qs) (all of at most 32 bases) are counted on
    // the matrix cores on clean waves (n_qs: none): three-class operands of
    // one word, four strands per column tile, dm_b[(2 tile + K step) * 64 +
    // lane], dm_t[32 tile + column] = L - k - nA (the exact hit bound)
    const uint4 *dm_b;
    const float *dm_t;
    uint32_t dm_first;
    // dense strands [dense_seam, n_qs) are those the encoding-3 variants may
    // count on the matrix cores; the dense strands come by L descending on
    // either side of the seam, so the VALU dense kernel runs each side in a
    // launch of its own: strands [dense_begin, dense_end), and with
    // dense_unclean only the waves that are not clean (those the matrix
    // kernel leaves out)
    uint32_t dense_seam;
    uint32_t dense_begin, dense_end;
    uint32_t dense_unclean;
    // overhang kernel: pieces per wave for the strand with the widest clip
    // (64 / (2 C) lanes each, at least 1); 0 = no strand can overhang
    uint32_t edge_pmin;
    // indexed mode: per-strand seed data, seed_ncfg tables (in device
    // memory), the masked centre length of every seed
    const SeedInfo *seed_info;
    const SeedTable *seed_tab;
    uint32_t seed_ncfg;
    uint32_t seed_mask;
    // count+digest sink, kStripes slots per query (see kStripes)
    unsigned long long *q_count;
    unsigned long long *q_digest;
};

// A scan-kernel launch recorded instead of issued (the launch functions'
// plan mode): kernel, grid, block, dynamic LDS and its one argument.
struct ScanLaunch {
    const void *func;
    dim3 grid, block;
    uint32_t lds;
    ScanArgs args;
};

}  // namespace ifa
