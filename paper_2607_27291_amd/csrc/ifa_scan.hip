// ifa_scan.hip -- gfx950 kernels of the brute-force gapless scan.
//
// Brute-force mode tests every start position of the reference against every
// query (Methods, "Algorithm Design"). The paper's CPU kernel compares one
// query base against 32 consecutive reference positions per vector step and
// keeps per-lane substitution and N ("clip") counters, stopping once every
// lane is past a threshold (Methods, "SIMD Optimization"). Here the reference
// is held as 2-bit bit planes and each GPU lane owns W consecutive window
// starts (W = 32: one plane word; W = 16: half a word).
//
// scan_filter_kernel (the hot loop), for the query strands predicted sparse:
//   * the lane loads plane words w and w+1 and forms, once, the W funnel
//     shifts (v_alignbit_b32) that give each of its windows' first 32 bases
//     as one word per plane; they are shared by every query and strand;
//   * per query strand, a window's mismatches over its first min(L, 32)
//     bases are popcount((qh ^ rh) | (ql ^ rl) | qn): two v_bitop3_b32 and
//     one v_bcnt_u32_b32, folded over the lane's windows with v_min3_u32.
//     Strands come sorted by L descending and the cached slices are masked in
//     place when L drops below 32, so query bits past L (zero) never differ.
//     A window can be a hit only if this count is <= k. When no window
//     passes (almost always), the lane is done with this query strand: the
//     paper's early exit, taken per 32 bases;
//   * waves whose first bases hold an N (rare) skip the filter and list
//     every strand for the resolve kernel, which applies the N rule;
//   * a wave with a candidate window appends one work item per batch of 32
//     query strands to a work list.
// scan_resolve_kernel: one wave per work item re-runs the filter for the
//   listed strands and runs the exact test on candidate lanes.
// scan_dense_kernel: query strands predicted to have candidates in most
//   waves skip the list; every lane resolves them directly.
// The exact test walks every query word and applies the N rule, piece ends
// and chunk ownership; hits go to records or to a per-query count+digest.
//
// Variants (template parameters, chosen by the autotuner): windows per lane
// W, query strands per filter iteration QU, and workgroup size.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <vector>
#include <mutex>
#include <type_traits>

#include "ifa_dev.h"

namespace ifa {

// Read-only data addressed uniformly by a wave is read through the constant
// address space so it becomes scalar loads into SGPRs.
#define IFA_CONST __attribute__((address_space(4)))

template <class T>
__device__ __forceinline__ const IFA_CONST T *as_const(const T *p)
{
    return (const IFA_CONST T *)(p);
}

// Three-input bitwise op (v_bitop3_b32): bit i of the result is bit
// (a_i << 2 | b_i << 1 | c_i) of the truth table.
#define IFA_XOR_OR 0xBEu   // (a ^ b) | c
#define IFA_OR_XOR 0xF6u   // a | (b ^ c)

__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s)
{
    // bits [s, s+32) of the 64-bit value hi:lo
    return __builtin_amdgcn_alignbit(hi, lo, s);
}

__device__ __forceinline__ uint32_t low_mask(uint32_t n)
{
    // n low bits set, n in [0, 32]
    return n >= 32u ? 0xffffffffu : ((1u << n) - 1u);
}

__device__ __forceinline__ uint64_t splitmix_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A query strand descriptor, unpacked from one 32-byte scalar load.
struct QS {
    uint32_t qid, len, strand, nw, k, maxn, woff, qh, ql, qn, thr;
};

__device__ __forceinline__ QS load_qs(const ScanArgs &a, uint32_t q)
{
    const IFA_CONST uint32_t *r = as_const(reinterpret_cast<const uint32_t *>(a.qs)) + 8u * q;
    const uint32_t r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
    const uint32_t r4 = r[4], r5 = r[5], r6 = r[6], r7 = r[7];
    QS d;
    d.qid = r0;
    d.len = r1 & 0xffffu;
    d.strand = (r1 >> 16) & 0xffu;
    d.nw = r1 >> 24;
    d.k = r2 & 0xffffu;
    d.maxn = r2 >> 16;
    d.woff = r3;
    d.qh = r4;
    d.ql = r5;
    d.qn = r6;
    d.thr = r7;
    return d;
}

// Hash of one hit for the count+digest sink: SplitMix64 output finaliser of
// ((contig << 32) | pos) ^ (aux << 45), aux = strand | m << 1 | n_ref << 10.
__device__ __forceinline__ uint64_t hit_hash(uint32_t contig, uint32_t pos, uint32_t strand,
                                             uint32_t m, uint32_t nref)
{
    const uint64_t key = ((uint64_t)contig << 32) | pos;
    const uint64_t aux = (uint64_t)strand | ((uint64_t)m << 1) | ((uint64_t)nref << 10);
    return splitmix_fin(key ^ (aux << 45));
}

// Index of the piece holding chunk position p (pieces sorted by start).
__device__ __forceinline__ uint32_t find_piece(const ScanArgs &a, uint64_t p)
{
    uint32_t lo = 0, hi = a.n_pieces;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (a.pieces[mid].start <= p) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void write_record(const ScanArgs &a, unsigned long long slot,
                                             const QS &d, uint32_t contig, uint32_t pos,
                                             uint32_t m, uint32_t nref)
{
    if (slot < a.hit_cap) {
        uint4 rec;
        rec.x = d.qid;
        rec.y = contig;
        rec.z = pos;
        rec.w = d.strand | (nref << 8) | (m << 16);
        a.hits[slot] = rec;
    }
}

// Per-lane state: the lane's W windows start at 32w + off.
struct Lane {
    uint32_t w, off;
    bool active;
    int plain;            // -1 unknown; 1: no N, piece end, carried prefix or chunk
                          // tail among the bases its windows can touch
    uint32_t h0, h1, l0, l1, n0, n1;
};

__device__ __forceinline__ bool lane_is_plain(const ScanArgs &a, const Lane &ln)
{
    const uint64_t first = 32ull * ln.w + ln.off;
    // windows start at first .. first + W - 1 and span up to lmax bases
    const uint64_t last = first + 31u + a.lmax;   // >= last base touched, W <= 32
    if (first < (uint64_t)a.own_from || last >= a.chunk_len) return false;
    const uint32_t wlast = (uint32_t)(last >> 5);
    uint32_t acc = 0;
    for (uint32_t x = ln.w; x <= wlast; x++) acc |= a.nm[x] | a.em[x];
    return acc == 0u;
}

// Exact test, any lane: one window at a time, every query word, N rule, piece
// ends, chunk ownership and tail. Records are written here (one atomic slot
// per hit: these lanes are rare); count+digest accumulates into cnt/dig.
template <int W>
__device__ void exact_serial(const ScanArgs &a, const QS &d, const Lane &ln, uint32_t &cnt,
                             uint64_t &dig)
{
    const uint32_t L = d.len;
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    const uint32_t w = ln.w;
#pragma unroll 1
    for (uint32_t b = ln.off; b < ln.off + (uint32_t)W; b++) {
        const uint64_t p = 32ull * w + b;
        if (p + L > a.chunk_len) break;
        if (p + L - 1 < (uint64_t)a.own_from) continue;
        uint32_t m = 0, nref = 0, ends = 0;
        for (uint32_t t = 0; t < d.nw; t++) {
            const uint32_t i0 = 32u * t;
            const uint32_t lmask = low_mask(L - i0);
            const uint32_t emask = (L - 1 > i0) ? low_mask(L - 1 - i0) : 0u;
            const uint32_t x = w + t;
            const uint32_t rh = funnel(a.hi[x + 1], a.hi[x], b);
            const uint32_t rl = funnel(a.lo[x + 1], a.lo[x], b);
            const uint32_t rn = funnel(a.nm[x + 1], a.nm[x], b);
            const uint32_t re = funnel(a.em[x + 1], a.em[x], b);
            const uint32_t qh = qw[3 * t], ql = qw[3 * t + 1], qn = qw[3 * t + 2];
            const uint32_t diff = (qh ^ rh) | (ql ^ rl) | qn;
            ends |= re & emask;
            if (a.policy == kNSeparate)
                m += __popc(diff & ~rn & lmask);
            else
                m += __popc((diff | rn) & lmask);
            nref += __popc(rn & lmask);
        }
        if (ends) continue;
        if (m > d.k) continue;
        if (a.policy == kNSeparate && nref > d.maxn) continue;
        const Piece pc = a.pieces[find_piece(a, p)];
        const uint32_t pos = (uint32_t)(pc.contig_off + (p - pc.start));
        if (a.sink == kSinkRecords) {
            write_record(a, atomicAdd(a.hit_count, 1ull), d, pc.contig, pos, m, nref);
        } else {
            cnt += 1;
            dig += hit_hash(pc.contig, pos, d.strand, m, nref);
        }
    }
}

// Exact test of a plain lane: no N, no piece end, every window owned and
// inside the chunk, all W windows in one piece. Word 0 comes from the lane's
// cached plane words; later query words only for windows still within k.
// kWrite = false: count (and hash) the hits; kWrite = true: write records to
// slots slot, slot + 1, ... in window order.
template <int W, bool kWrite>
__device__ void exact_plain(const ScanArgs &a, const QS &d, const Lane &ln, uint32_t contig,
                            uint32_t pos0, uint32_t &cnt, uint64_t &dig,
                            unsigned long long slot)
{
    const uint32_t L = d.len;
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    const uint32_t lmask0 = low_mask(L);
    uint32_t h2 = 0, l2 = 0, qh1 = 0, ql1 = 0, qn1 = 0, lmask1 = 0;
    if (d.nw >= 2) {
        h2 = a.hi[ln.w + 2];
        l2 = a.lo[ln.w + 2];
        qh1 = qw[3];
        ql1 = qw[4];
        qn1 = qw[5];
        lmask1 = low_mask(L - 32u);
    }
#pragma unroll 1
    for (uint32_t b = 0; b < (uint32_t)W; b++) {
        const uint32_t s = ln.off + b;
        uint32_t diff = __builtin_amdgcn_bitop3_b32(funnel(ln.h1, ln.h0, s), d.qh, d.qn, IFA_XOR_OR);
        diff = __builtin_amdgcn_bitop3_b32(diff, funnel(ln.l1, ln.l0, s), d.ql, IFA_OR_XOR);
        uint32_t m = __popc(diff & lmask0);
        if (m <= d.k && d.nw >= 2) {
            uint32_t d1 = __builtin_amdgcn_bitop3_b32(funnel(h2, ln.h1, s), qh1, qn1, IFA_XOR_OR);
            d1 = __builtin_amdgcn_bitop3_b32(d1, funnel(l2, ln.l1, s), ql1, IFA_OR_XOR);
            m += __popc(d1 & lmask1);
            for (uint32_t t = 2; t < d.nw && m <= d.k; t++) {
                const uint32_t x = ln.w + t;
                const uint32_t rh = funnel(a.hi[x + 1], a.hi[x], s);
                const uint32_t rl = funnel(a.lo[x + 1], a.lo[x], s);
                const uint32_t dt = (qw[3 * t] ^ rh) | (qw[3 * t + 1] ^ rl) | qw[3 * t + 2];
                m += __popc(dt & low_mask(L - 32u * t));
            }
        }
        if (m <= d.k) {
            if (kWrite) {
                write_record(a, slot, d, contig, pos0 + b, m, 0u);
                slot++;
            } else {
                cnt += 1;
                if (a.sink == kSinkCountDigest) dig += hit_hash(contig, pos0 + b, d.strand, m, 0u);
            }
        }
    }
}

// Wave-wide sums with DPP moves (no LDS round trips): an inclusive scan
// within each row of 16 lanes (row_shr 1, 2, 4, 8), then row 0's total is
// broadcast into row 1 and row 2's into row 3 (row_bcast:15), then lane 31's
// into rows 2 and 3 (row_bcast:31); lane 63 ends with the wave's total.
// Lanes whose DPP source is out of range or masked read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_get(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void dpp_step(uint32_t &c, uint32_t &lo, uint32_t &hi)
{
    const uint32_t tc = dpp_get<CTRL, ROWS>(c);
    const uint32_t tl = dpp_get<CTRL, ROWS>(lo);
    const uint32_t th = dpp_get<CTRL, ROWS>(hi);
    const uint32_t nl = lo + tl;
    hi += th + (nl < lo ? 1u : 0u);
    lo = nl;
    c += tc;
}

// Sum cnt / dig over the wave and add them once, to stripe `stripe` of the
// query's count+digest accumulators. Called by all 64 lanes.
__device__ __forceinline__ void wave_add_stats(const ScanArgs &a, uint32_t qid, uint32_t cnt,
                                               uint64_t dig, uint32_t stripe)
{
    if (!__any(cnt != 0u)) return;
    uint32_t lo = (uint32_t)dig, hi = (uint32_t)(dig >> 32);
    dpp_step<0x111, 0xf>(cnt, lo, hi);   // row_shr:1
    dpp_step<0x112, 0xf>(cnt, lo, hi);   // row_shr:2
    dpp_step<0x114, 0xf>(cnt, lo, hi);   // row_shr:4
    dpp_step<0x118, 0xf>(cnt, lo, hi);   // row_shr:8
    dpp_step<0x142, 0xa>(cnt, lo, hi);   // row_bcast:15 into rows 1, 3
    dpp_step<0x143, 0xc>(cnt, lo, hi);   // row_bcast:31 into rows 2, 3
    const uint32_t tc = (uint32_t)__builtin_amdgcn_readlane((int)cnt, 63);
    const uint32_t tl = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
    const uint32_t th = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
    if ((threadIdx.x & 63u) == 0u) {
        const uint32_t slot = qid * kStripes + stripe % kStripes;
        atomicAdd(&a.q_count[slot], (unsigned long long)tc);
        atomicAdd(&a.q_digest[slot], ((unsigned long long)th << 32) | tl);
    }
}

// One query strand against the lane's windows after the filter: exact test
// where `cand`, then (count+digest) a wave-wide sum added once per wave to
// stripe `stripe` of the query's accumulators. Called by all 64 lanes.
template <int W>
__device__ __forceinline__ void resolve(const ScanArgs &a, const QS &d, Lane &ln, bool cand,
                                        uint32_t stripe)
{
    const bool mine = ln.active && cand;
    if (!__any(mine)) return;
    uint32_t cnt = 0;
    uint64_t dig = 0;
    if (mine) {
        if (ln.plain < 0) ln.plain = lane_is_plain(a, ln) ? 1 : 0;
        if (ln.plain) {
            const uint64_t first = 32ull * ln.w + ln.off;
            const Piece pc = a.pieces[find_piece(a, first)];
            const uint32_t pos0 = (uint32_t)(pc.contig_off + (first - pc.start));
            exact_plain<W, false>(a, d, ln, pc.contig, pos0, cnt, dig, 0ull);
            if (a.sink == kSinkRecords && cnt) {
                unsigned long long slot = atomicAdd(a.hit_count, (unsigned long long)cnt);
                uint32_t c2 = 0;
                uint64_t d2 = 0;
                exact_plain<W, true>(a, d, ln, pc.contig, pos0, c2, d2, slot);
            }
        } else {
            exact_serial<W>(a, d, ln, cnt, dig);
        }
    }
    if (a.sink == kSinkCountDigest) wave_add_stats(a, d.qid, cnt, dig, stripe);
}

// Minimum over the lane's W windows of the filter count for one query strand
// (hot loop: slices cached in registers, already masked to the strand's first
// min(L, 32) bases; the wave holds no N).
template <int W>
__device__ __forceinline__ uint32_t filter_min(const uint32_t (&sh)[W], const uint32_t (&sl)[W],
                                               const QS &d)
{
    uint32_t mn = 0xffffffffu;
#pragma unroll
    for (int b = 0; b < W; b++) {
        uint32_t diff = __builtin_amdgcn_bitop3_b32(sh[b], d.qh, d.qn, IFA_XOR_OR);
        diff = __builtin_amdgcn_bitop3_b32(diff, sl[b], d.ql, IFA_OR_XOR);
        mn = min(mn, (uint32_t)__popc(diff));
    }
    return mn;
}

// The filter decision formed from the lane's plane words (cold paths), over
// the first min(L, 32 nw) bases, nw = 1 or 2 (the prefix words the strand's
// three-class matrix tile filters on). N positions: under N_SEPARATE they are
// left out of the count, and a window whose N count there already exceeds
// maxN is pushed past any threshold; under N_AS_MISMATCH they are mismatches.
template <int W>
__device__ __forceinline__ bool filter_cand_words(const ScanArgs &a, const QS &d, const Lane &ln,
                                                  uint32_t nw)
{
    const bool two = nw >= 2u && d.len > 32u;
    if (!two && d.thr >= 32u) return true;
    const uint32_t lmask = low_mask(d.len), lmask1 = two ? low_mask(d.len - 32u) : 0u;
    uint32_t h2 = 0, l2 = 0, n2 = 0, qh1 = 0, ql1 = 0, qn1 = 0;
    if (two) {
        const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
        h2 = a.hi[ln.w + 2];
        l2 = a.lo[ln.w + 2];
        n2 = a.nm[ln.w + 2];
        qh1 = qw[3];
        ql1 = qw[4];
        qn1 = qw[5];
    }
    uint32_t mn = 0xffffffffu;
#pragma unroll 4
    for (int b = 0; b < W; b++) {
        const uint32_t s = ln.off + (uint32_t)b;
        uint32_t diff = __builtin_amdgcn_bitop3_b32(funnel(ln.h1, ln.h0, s), d.qh, d.qn, IFA_XOR_OR);
        diff = __builtin_amdgcn_bitop3_b32(diff, funnel(ln.l1, ln.l0, s), d.ql, IFA_OR_XOR);
        const uint32_t rn = funnel(ln.n1, ln.n0, s) & lmask;
        diff &= lmask;
        uint32_t d1 = 0, rn1 = 0;
        if (two) {
            d1 = __builtin_amdgcn_bitop3_b32(funnel(h2, ln.h1, s), qh1, qn1, IFA_XOR_OR);
            d1 = __builtin_amdgcn_bitop3_b32(d1, funnel(l2, ln.l1, s), ql1, IFA_OR_XOR) & lmask1;
            rn1 = funnel(n2, ln.n1, s) & lmask1;
        }
        if (a.policy == kNSeparate) {
            const uint32_t over = __popc(rn) + __popc(rn1) > d.maxn ? 512u : 0u;
            mn = min(mn, (uint32_t)(__popc(diff & ~rn) + __popc(d1 & ~rn1)) + over);
        } else {
            mn = min(mn, (uint32_t)(__popc(diff | rn) + __popc(d1 | rn1)));
        }
    }
    return mn <= d.thr;
}

// Prefix words (1 or 2) the strand at sparse index q filters on: those of its
// three-class matrix column tile; 1 for dense strands.
__device__ __forceinline__ uint32_t strand_filter_words(const ScanArgs &a, uint32_t q)
{
    return q < a.n_sparse ? a.mq3_w[q >> 2] & 0xffu : 1u;
}

// Lane state of filter-grid lane `gl` (relative to w_begin).
template <int W>
__device__ __forceinline__ Lane make_lane(const ScanArgs &a, uint32_t gl)
{
    constexpr uint32_t kLanesPerWord = 32 / W;
    Lane ln;
    ln.w = a.w_begin + gl / kLanesPerWord;
    ln.off = (gl % kLanesPerWord) * (uint32_t)W;
    ln.active = ln.w < a.w_end;
    ln.plain = -1;
    if (!ln.active) ln.w = a.w_begin;    // inactive lanes read valid words, report nothing
    ln.h0 = a.hi[ln.w];
    ln.h1 = a.hi[ln.w + 1];
    ln.l0 = a.lo[ln.w];
    ln.l1 = a.lo[ln.w + 1];
    ln.n0 = a.nm[ln.w];
    ln.n1 = a.nm[ln.w + 1];
    return ln;
}

// Mask the cached slices to the first L bases (L < 32). Sparse strands come
// sorted by L descending, so masks only ever shrink and can be applied in
// place: bases past L then never differ from the zero query bits there.
template <int W>
__device__ __forceinline__ void mask_slices(uint32_t (&sh)[W], uint32_t (&sl)[W], uint32_t L)
{
    const uint32_t m = low_mask(L);
#pragma unroll
    for (int b = 0; b < W; b++) {
        sh[b] &= m;
        sl[b] &= m;
    }
}

// Filter the sparse query strands; one work item per (wave, batch of 32
// strands) that has a candidate window in any lane.
template <int W, int QU>
__device__ __forceinline__ void filter_lane(const ScanArgs &a, const Lane &ln, uint32_t wave)
{
    uint32_t sh[W], sl[W];
#pragma unroll
    for (int b = 0; b < W; b++) {
        sh[b] = funnel(ln.h1, ln.h0, ln.off + (uint32_t)b);
        sl[b] = funnel(ln.l1, ln.l0, ln.off + (uint32_t)b);
    }
    uint32_t cur_len = 32;      // slices hold this many bases (wave-uniform)
    const uint32_t n = a.n_sparse;
    for (uint32_t qb = 0; qb < n; qb += 32) {
        const uint32_t nb = min(32u, n - qb);
        uint32_t pending = 0;   // wave-uniform
        uint32_t j = 0;
        if (QU == 2) {
            for (; j + 1 < nb; j += 2) {
                const QS d0 = load_qs(a, qb + j);
                const QS d1 = load_qs(a, qb + j + 1);
                if (d0.len < cur_len) {
                    mask_slices<W>(sh, sl, d0.len);
                    cur_len = d0.len;
                }
                const bool c0 = d0.thr >= 32u ||
                    filter_min<W>(sh, sl, d0) <= d0.thr;
                if (d1.len < cur_len) {
                    mask_slices<W>(sh, sl, d1.len);
                    cur_len = d1.len;
                }
                const bool c1 = d1.thr >= 32u ||
                    filter_min<W>(sh, sl, d1) <= d1.thr;
                if (__any(ln.active && c0)) pending |= 1u << j;
                if (__any(ln.active && c1)) pending |= 2u << j;
            }
        }
        for (; j < nb; j++) {
            const QS d = load_qs(a, qb + j);
            if (d.len < cur_len) {
                mask_slices<W>(sh, sl, d.len);
                cur_len = d.len;
            }
            const bool c = d.thr >= 32u ||
                filter_min<W>(sh, sl, d) <= d.thr;
            if (__any(ln.active && c)) pending |= 1u << j;
        }
        if (pending && (threadIdx.x & 63u) == 0u) {
            const unsigned int idx = atomicAdd(a.work_count, 1u);
            if (idx < a.work_cap) {
                WorkItem it;
                it.wave = wave;
                it.qb = qb;
                it.pending = pending;
                it.pad = 0;
                a.work[idx] = it;
            }
        }
    }
}

// Work items for a wave that holds an N: every strand of the batch at qb is
// listed, as items of list_per strands so that different resolve waves share
// the batch (these items carry all their strands, unlike filtered ones).
__device__ __forceinline__ void list_batch(const ScanArgs &a, uint32_t wave, uint32_t qb)
{
    const uint32_t nb = min(32u, a.n_sparse - qb);
    const uint32_t all = nb == 32u ? 0xffffffffu : ((1u << nb) - 1u);
    const uint32_t per = a.list_per;
    const uint32_t items = (nb + per - 1u) / per;
    const unsigned int idx = atomicAdd(a.work_count, items);
    for (uint32_t p = 0; p < items; p++) {
        if (idx + p < a.work_cap) {
            WorkItem it;
            it.wave = wave;
            it.qb = qb;
            it.pending = all & (((1u << per) - 1u) << (per * p));
            it.pad = 0;
            a.work[idx + p] = it;
        }
    }
}

template <int W, int QU, int WG>
__global__ __launch_bounds__(WG) void scan_filter_kernel(ScanArgs a)
{
    const uint32_t gl = blockIdx.x * WG + threadIdx.x;
    const Lane ln = make_lane<W>(a, gl);
    const uint32_t wave = gl >> 6;
    // Does any base the filter reads for this lane hold an N? Words w and
    // w+1 cover the first 32 bases of all of the lane's windows. Such waves
    // are rare; they skip the filter and list every strand for the resolve
    // kernel, whose filter applies the N rule (keeping that rule out of this
    // kernel saves ~30 VGPRs of occupancy for every other wave).
    const bool lane_n = ln.active && ((ln.n0 | ln.n1) != 0u);
    if (__any(lane_n)) {
        if ((threadIdx.x & 63u) == 0u) {
            atomicAdd(a.skip_count, 1u);
            for (uint32_t qb = 0; qb < a.n_sparse; qb += 32) list_batch(a, wave, qb);
        }
        return;
    }
    filter_lane<W, QU>(a, ln, wave);
}

// ---------------------------------------------------------------------------
// Matrix-core filter (gfx950 fp4 MFMA).
//
// The filter count of window p and strand s is L32 minus the number of
// matches over the first L32 = min(L, 32) bases, and the match count is a
// dense contraction of one-hot codes:
//   matches(p, s) = sum over j < L32, classes b of [S[p+j] = b] [Q_s[j] = b]
// (a query N has no class, so it never matches). Windows are taken in groups
// of 16 consecutive starts; group g covers the 48-base segment S[16g, 16g+48)
// and the 16 shifts r of a strand become 16 columns of a banded operand:
//   B[(i, b), (s, r)] = [Q_s[i - r] = b] for 0 <= i - r < L32, else 0,
// so matches(16g + r, s) = sum over i < 48, b of A[g, (i, b)] B[(i, b), (s, r)]
// with A[g, (i, b)] = [S[16g + i] = b]: a (groups x 192) by (192 x 16
// strands) product in e2m1 (1.0 or 0), exact in the fp32 accumulator.
//
// One wave covers the 1024 window starts of a filter wave (64 lanes x 16):
// two 32-group A tiles, each 3 K-steps of v_mfma_scale_f32_32x32x64_f8f6f4
// (32 groups x 64 K per step). Operand layout of that instruction: lane l
// holds row (A) or column (B) l % 32 and K elements 32 (l / 32) + e, e < 32,
// element e in bits 4e..4e+3 of the lane's four registers; lane l of D holds
// column l % 32, rows 8 (i / 4) + 4 (l / 32) + i % 4 in its 16 registers.
// Here K step t, half h = l / 32 covers segment bases 16t + 8h + o, o < 8,
// and element e = 8b + o: register b holds class b's one-hot nibbles of the
// lane's 8 bases. The B operand (two strands x 16 shifts per 32-column tile,
// built on the host in this order) and each column's required match count
// come from mq_b / mq_t. A window may be a hit only if its matches reach the
// column's count; per tile the wave takes the maximum over its rows.
// ---------------------------------------------------------------------------

typedef int ifa_v8i __attribute__((ext_vector_type(8)));
typedef float ifa_v16f __attribute__((ext_vector_type(16)));

// byte x -> bit 4o+1 (the e2m1 code of 1.0 in nibble o) for each set bit o
struct SpreadTable {
    uint32_t v[256];
};
constexpr SpreadTable make_spread_table()
{
    SpreadTable t{};
    for (uint32_t x = 0; x < 256; x++) {
        uint32_t s = 0;
        for (uint32_t o = 0; o < 8; o++)
            if ((x >> o) & 1u) s |= 2u << (4u * o);
        t.v[x] = s;
    }
    return t;
}
__device__ const SpreadTable kSpread = make_spread_table();

// The lane's A operand of one K step: one-hot nibbles of 8 bases whose hi and
// lo bits are the low bytes of hb, lb. Register b = class b = 2 hi + lo.
__device__ __forceinline__ ifa_v8i onehot_operand(uint32_t hb, uint32_t lb)
{
    const uint32_t sh = kSpread.v[hb & 0xffu], sl = kSpread.v[lb & 0xffu];
    const uint32_t m = 0x22222222u;
    ifa_v8i r = {};
    r[0] = (int)(~sh & ~sl & m);
    r[1] = (int)(~sh & sl & m);
    r[2] = (int)(sh & ~sl & m);
    r[3] = (int)(sh & sl & m);
    return r;
}

// The 8 XCDs of the chip take workgroups round-robin by linear workgroup id,
// and each has its own L2. Filter waves read one 128-byte line past their own
// (the first line of the next wave's words), so neighbouring waves on
// different XCDs fetch that line twice from HBM. With gridDim.x a multiple of
// 8 (the host rounds it), the x index is permuted so that each XCD holds a
// contiguous run of x indices: xcd * (gridDim.x / 8) + the block's rank
// within its XCD; the workgroups of one XCD then walk adjacent waves.
__device__ __forceinline__ uint32_t xcd_local_x()
{
    const uint32_t g = gridDim.x;
    if (g % 8u != 0u) return blockIdx.x;
    const uint32_t lin = blockIdx.x + blockIdx.y * g;   // the dispatcher's order
    return (lin % 8u) * (g / 8u) + blockIdx.x / 8u;
}

__device__ __forceinline__ ifa_v16f mfma_fp4(const ifa_v8i &a, const ifa_v8i &b, const ifa_v16f &c)
{
    // cbsz = blgp = 4: both operands e2m1; E8M0 scales 127 = 1.0
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

// Grid: x = workgroups sharing one batch of 32 sparse strands (16 column
// tiles), y = batch. A workgroup copies its batch's B operands, required
// counts and the spread table into LDS once, then its waves walk filter waves
// blockIdx.x * (WG / 64) + wave, stepping by gridDim.x * (WG / 64). Dynamic
// LDS: mq_lds_bytes(tiles of the batch).
template <int WG>
__global__ __launch_bounds__(WG) void scan_filter_mfma_kernel(ScanArgs a)
{
    extern __shared__ uint4 lds[];
    const uint32_t qb = 32u * (a.batch0 + blockIdx.y);
    const uint32_t n_tiles = (a.n_sparse + 1u) >> 1;
    const uint32_t t0 = qb >> 1, tn = min(n_tiles, t0 + 16u) - t0;   // tiles of the batch
    uint4 *sb = lds;                                                 // [tn][3][64]
    float *st = reinterpret_cast<float *>(lds + 192u * tn);          // [tn][32]
    uint32_t *sp = reinterpret_cast<uint32_t *>(st + 32u * tn);      // [256]
    for (uint32_t i = threadIdx.x; i < 192u * tn; i += WG) sb[i] = a.mq_b[192u * t0 + i];
    for (uint32_t i = threadIdx.x; i < 32u * tn; i += WG) st[i] = a.mq_t[32u * t0 + i];
    for (uint32_t i = threadIdx.x; i < 256u; i += WG) sp[i] = kSpread.v[i];
    __syncthreads();

    const uint32_t l = threadIdx.x & 63u;
    const uint32_t g = l & 31u, h = l >> 5;
    const uint32_t last = (uint32_t)((a.chunk_len + 31) >> 5) + kPadWords - 1;
    const uint32_t n_waves = (a.w_end - a.w_begin + 31u) >> 5;
    const uint32_t stride = gridDim.x * (WG / 64u);
    const ifa_v16f zero = {};
    for (uint32_t wave = xcd_local_x() * (WG / 64u) + (threadIdx.x >> 6); wave < n_waves;
         wave += stride) {
        // lane l of a filter wave stands for plane word w0 + l / 2 (16
        // windows); the N test and the work items are those of the VALU filter
        const uint32_t w0 = a.w_begin + 32u * wave;
        const uint32_t lw = w0 + (l >> 1);
        bool lane_n = false;
        if (lw < a.w_end) lane_n = (a.nm[lw] | a.nm[min(lw + 1u, last)]) != 0u;
        if (__any(lane_n)) {
            if (l == 0u) {
                if (a.batch0 + blockIdx.y == 0) atomicAdd(a.skip_count, 1u);
                list_batch(a, wave, qb);
            }
            continue;
        }
        // A operands: tile u holds groups 32u + g (window starts 512u + 16g)
        ifa_v8i A[2][3];
#pragma unroll
        for (int u = 0; u < 2; u++) {
            const uint32_t wa = min(w0 + 16u * u + (g >> 1), last);
            const uint32_t wb = min(wa + 1u, last);
            const uint64_t hh = ((uint64_t)a.hi[wb] << 32) | a.hi[wa];
            const uint64_t ll = ((uint64_t)a.lo[wb] << 32) | a.lo[wa];
#pragma unroll
            for (int t = 0; t < 3; t++) {
                const uint32_t x = 16u * (g & 1u) + 16u * t + 8u * h;   // < 64
                const uint32_t s1 = sp[(uint32_t)(hh >> x) & 0xffu];
                const uint32_t s0 = sp[(uint32_t)(ll >> x) & 0xffu];
                const uint32_t m = 0x22222222u;
                ifa_v8i r = {};
                r[0] = (int)(~s1 & ~s0 & m);
                r[1] = (int)(~s1 & s0 & m);
                r[2] = (int)(s1 & ~s0 & m);
                r[3] = (int)(s1 & s0 & m);
                A[u][t] = r;
            }
        }
        uint32_t pending = 0;   // wave-uniform
        for (uint32_t nt = 0; nt < tn; nt++) {
            ifa_v8i B[3];
#pragma unroll
            for (int t = 0; t < 3; t++) {
                const uint4 v = sb[(3u * nt + (uint32_t)t) * 64u + l];
                B[t] = ifa_v8i{(int)v.x, (int)v.y, (int)v.z, (int)v.w, 0, 0, 0, 0};
            }
            const float need = st[32u * nt + g];
            ifa_v16f d0 = mfma_fp4(A[0][0], B[0], zero);
            ifa_v16f d1 = mfma_fp4(A[1][0], B[0], zero);
            d0 = mfma_fp4(A[0][1], B[1], d0);
            d1 = mfma_fp4(A[1][1], B[1], d1);
            d0 = mfma_fp4(A[0][2], B[2], d0);
            d1 = mfma_fp4(A[1][2], B[2], d1);
            // match counts are non-negative floats, which order as their bits
            uint32_t mx = 0;
#pragma unroll
            for (int i = 0; i < 16; i++)
                mx = max(max(__float_as_uint(d0[i]), __float_as_uint(d1[i])), mx);
            const uint64_t m = __ballot(__uint_as_float(mx) >= need);
            if (m & 0x0000ffff0000ffffull) pending |= 1u << (2u * nt);
            if (m & 0xffff0000ffff0000ull) pending |= 2u << (2u * nt);
        }
        if (pending && l == 0u) {
            const unsigned int idx = atomicAdd(a.work_count, 1u);
            if (idx < a.work_cap) {
                WorkItem it;
                it.wave = wave;
                it.qb = qb;
                it.pending = pending;
                it.pad = 0;
                a.work[idx] = it;
            }
        }
    }
}

// LDS bytes of the matrix-core filter for a batch of `tiles` column tiles.
static uint32_t mq_lds_bytes(uint32_t tiles)
{
    return tiles * (192u * 16u + 32u * 4u) + 256u * 4u;
}

// ---------------------------------------------------------------------------
// Matrix-core filter, three-class form (fewer K steps).
//
// For a reference base that is not N, [S = A] = 1 - [S = C] - [S = G] -
// [S = T], so with nA the number of A bases among the first L32 query bases
//   matches(p, s) = nA + sum over j < L32, b in {C, G, T} of [S[p+j] = b] w
// where w = +1 if Q_s[j] = b, -1 if Q_s[j] = A, 0 if Q_s[j] is another base
// or N. Three indicator classes per base instead of four: groups of 8
// windows read a 39-base segment, 117 K values, which fit two K steps of 64
// (against three for the four-class form with 16 windows per group), so
// every K element the instruction multiplies is used.
//
// Tile: 32 groups x 8 windows = 256 window starts; four tiles per filter wave.
// Column tile: 4 strands x 8 shifts. K layout: the segment's 8-base blocks
// k = 0..4 each give three indicator words (class C, G, T; nibble o = base
// 8k + o, e2m1 1.0 or 0); slot z = 8t + 4h + d (K step t, lane half h,
// register d) holds block z / 3, class z % 3; slot 15 meets only zero B
// entries. K step 0 thus holds blocks 0 and 1 in every class: a half-step
// tile (flag 0x100 in mq3_w) runs it alone and tests the window at shift r
// on its first 16 - r bases. A wave first writes the indicator words of its
// stream (m3_blocks blocks of 8 bases, three words each) to its own LDS
// area; the slots of lane (g, h) in tile u are words 3 (32u + g) + 4h + 8t
// + d. mq3_t holds the match count minus nA that a column needs.
// ---------------------------------------------------------------------------

// 8-base blocks a wave stages: its 1024 windows read up to base
// 1024 + 32 NW + 7 of its stream (block 132 + 4 (NW - 1) at most)
__host__ __device__ constexpr uint32_t m3_blocks(int nw) { return 136u + 4u * (uint32_t)(nw - 1); }

// NW: most prefix words (32 bases each) of the launch's column tiles; tile nt
// filters on mq3_w[nt] <= NW of them, each adding two K steps to its sums.
// The one-word form keeps four waves per SIMD with the pipeline's second set
// of accumulators (at most 128 VGPRs).
template <int WG, int NW>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(NW == 1 ? 4 : 1)))
void scan_filter_mfma3_kernel(ScanArgs a)
{
    constexpr uint32_t kBlocks = m3_blocks(NW), kWords = 3 * kBlocks;
    extern __shared__ uint4 lds[];
    const uint32_t qb = 32u * (a.batch0 + blockIdx.y);
    const uint32_t n_tiles = (a.n_sparse + 3u) >> 2;
    const uint32_t t0 = qb >> 2, tn = min(n_tiles, t0 + 8u) - t0;   // tiles of the batch
    uint4 *sb = lds;                                                // [tn][2 words][2][64]
    float *st = reinterpret_cast<float *>(lds + 256u * tn);         // [tn][32]
    uint32_t *sw = reinterpret_cast<uint32_t *>(st + 32u * tn);     // [8]
    uint32_t *sp = sw + 8;                                          // [256]
    uint32_t *flat = sp + 256u + (threadIdx.x >> 6) * kWords;       // this wave's words
    for (uint32_t i = threadIdx.x; i < 256u * tn; i += WG) sb[i] = a.mq3_b[256u * t0 + i];
    for (uint32_t i = threadIdx.x; i < 32u * tn; i += WG) st[i] = a.mq3_t[32u * t0 + i];
    for (uint32_t i = threadIdx.x; i < tn; i += WG) sw[i] = a.mq3_w[t0 + i];
    for (uint32_t i = threadIdx.x; i < 256u; i += WG) sp[i] = kSpread.v[i];
    __syncthreads();

    const uint32_t l = threadIdx.x & 63u;
    const uint32_t g = l & 31u, h = l >> 5;
    const uint32_t last = (uint32_t)((a.chunk_len + 31) >> 5) + kPadWords - 1;
    const uint32_t n_waves = (a.w_end - a.w_begin + 31u) >> 5;
    const uint32_t stride = gridDim.x * (WG / 64u);
    const ifa_v16f zero = {};
    // tiles of the batch that run the first K step alone: none, or all
    bool all_full = true, all_half = true;
    for (uint32_t i = 0; i < tn; i++) {
        const bool hf = (sw[i] >> 8) != 0u;
        all_full = all_full && !hf;
        all_half = all_half && hf;
    }
    // Lane j < kBlocks / 4 holds plane word j of a wave's stream (its four
    // 8-base blocks). A window filtered on NW prefix words reads the words of
    // its start .. start + NW, so the wave reads words w0 .. w0 + 31 + NW;
    // lane j <= ((w0 + 31 + NW) >> 5) - (w0 >> 5) (at most 3 lanes) also
    // holds the N flag of 32-word block (w0 >> 5) + j, so that any N the
    // wave's windows read (and possibly some they do not) sends the wave to
    // the exact path. The words of a lane's next wave are loaded before the
    // current wave's tiles run.
    static_assert(kBlocks % 4u == 0u && kBlocks / 4u <= 64u, "one plane word per lane");
    auto fetch = [&](uint32_t wv, uint32_t &ph, uint32_t &pl, uint32_t &pn) {
        const uint32_t w0 = a.w_begin + 32u * wv, w = min(w0 + l, last);
        ph = 0u;
        pl = 0u;
        pn = 0u;
        if (l < kBlocks / 4u) {
            ph = a.hi[w];
            pl = a.lo[w];
        }
        if (l <= ((w0 + 31u + (uint32_t)NW) >> 5) - (w0 >> 5)) pn = a.nflag[(w0 >> 5) + l];
    };
    uint32_t wave = xcd_local_x() * (WG / 64u) + (threadIdx.x >> 6);
    uint32_t nh = 0u, nl = 0u, nn = 0u;
    if (wave < n_waves) fetch(wave, nh, nl, nn);
    for (; wave < n_waves; wave += stride) {
        const uint32_t ch = nh, cl = nl, cn = nn;
        if (wave + stride < n_waves) fetch(wave + stride, nh, nl, nn);
        if (__any(cn != 0u)) {
            if (l == 0u) {
                if (a.batch0 + blockIdx.y == 0) atomicAdd(a.skip_count, 1u);
                list_batch(a, wave, qb);
            }
            continue;
        }
        // stage the indicator words of blocks 4j .. 4j + 3 (lane j)
        if (l < kBlocks / 4u) {
            const uint32_t m = 0x22222222u;
            uint32_t v[12];
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                const uint32_t s1 = sp[(ch >> (8u * q)) & 0xffu];
                const uint32_t s0 = sp[(cl >> (8u * q)) & 0xffu];
                v[3 * q] = ~s1 & s0 & m;           // C (hi 0, lo 1)
                v[3 * q + 1] = s1 & s0 & m;        // G (1, 1)
                v[3 * q + 2] = s1 & ~s0 & m;       // T (1, 0)
            }
            uint4 *dst = reinterpret_cast<uint4 *>(flat + 12u * l);
            dst[0] = make_uint4(v[0], v[1], v[2], v[3]);
            dst[1] = make_uint4(v[4], v[5], v[6], v[7]);
            dst[2] = make_uint4(v[8], v[9], v[10], v[11]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // word w of group g reads the segment from block g + 4w
        ifa_v8i A[NW][4][2];
#pragma unroll
        for (int w = 0; w < NW; w++)
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t *f = flat + 3u * (32u * u + g + 4u * w) + 4u * h;
#pragma unroll
                for (int t = 0; t < 2; t++)
                    A[w][u][t] = ifa_v8i{(int)f[8 * t], (int)f[8 * t + 1], (int)f[8 * t + 2],
                                         (int)f[8 * t + 3], 0, 0, 0, 0};
            }
        uint32_t pending = 0;   // wave-uniform
        // One-word batches whose tiles all run both K steps, or all the
        // first alone: a software pipeline over two sets of accumulators. The
        // p1 MFMAs of tile nt run while the p0 counts of tile nt are folded,
        // and the p0 MFMAs of tile nt + 1 while the p1 counts of tile nt are
        // folded, so that each wave keeps the matrix core busy during its own
        // fold.
        auto pipeline = [&](auto half_tag) {
            constexpr bool kHalf = decltype(half_tag)::value;
            auto ldB = [&](uint32_t nt, ifa_v8i &B0, ifa_v8i &B1, float &nd) {
                const uint4 v0 = sb[(4u * nt) * 64u + l];
                B0 = ifa_v8i{(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, 0, 0, 0, 0};
                if (!kHalf) {
                    const uint4 v1 = sb[(4u * nt + 1u) * 64u + l];
                    B1 = ifa_v8i{(int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w, 0, 0, 0, 0};
                }
                nd = st[32u * nt + g];
            };
            // the counts of row tiles 2p and 2p + 1 of a column tile
            auto counts = [&](int p, const ifa_v8i &B0, const ifa_v8i &B1, ifa_v16f &d0,
                              ifa_v16f &d1) {
                d0 = mfma_fp4(A[0][2 * p][0], B0, zero);
                d1 = mfma_fp4(A[0][2 * p + 1][0], B0, zero);
                if (!kHalf) {
                    d0 = mfma_fp4(A[0][2 * p][1], B1, d0);
                    d1 = mfma_fp4(A[0][2 * p + 1][1], B1, d1);
                }
            };
            auto mark = [&](uint32_t nt, float mx, float need) {
                const uint64_t m = __ballot(mx >= need);
#pragma unroll
                for (uint32_t q = 0; q < 4; q++)
                    if (m & (0x000000ff000000ffull << (8u * q))) pending |= 1u << (4u * nt + q);
            };
            ifa_v8i cB0 = {}, cB1 = {}, nB0 = {}, nB1 = {};
            float cneed, nneed;
            ifa_v16f a0, a1, b0, b1;
            ldB(0, cB0, cB1, cneed);
            counts(0, cB0, cB1, a0, a1);
            for (uint32_t nt = 0; nt + 1u < tn; nt++) {
                ldB(nt + 1u, nB0, nB1, nneed);
                counts(1, cB0, cB1, b0, b1);
                float mx = -1e30f;
#pragma unroll
                for (int i = 0; i < 16; i++) mx = fmaxf(fmaxf(a0[i], a1[i]), mx);
                counts(0, nB0, nB1, a0, a1);
#pragma unroll
                for (int i = 0; i < 16; i++) mx = fmaxf(fmaxf(b0[i], b1[i]), mx);
                mark(nt, mx, cneed);
                cB0 = nB0;
                cB1 = nB1;
                cneed = nneed;
                // the order above, interleaved: each MFMA followed by VALU
                // instructions of the fold that does not wait on it
                constexpr int kMfma = kHalf ? 4 : 8;
#pragma unroll
                for (int i = 0; i < kMfma; i++) {
                    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                    __builtin_amdgcn_sched_group_barrier(0x002, 32 / kMfma, 0);
                }
            }
            // the last tile: its p1 MFMAs beside the fold of its p0 counts
            counts(1, cB0, cB1, b0, b1);
            float mx = -1e30f;
#pragma unroll
            for (int i = 0; i < 16; i++) mx = fmaxf(fmaxf(a0[i], a1[i]), mx);
#pragma unroll
            for (int i = 0; i < 16; i++) mx = fmaxf(fmaxf(b0[i], b1[i]), mx);
            mark(tn - 1u, mx, cneed);
        };
        if (NW == 1 && all_full) {
            pipeline(std::false_type{});
        } else if (NW == 1 && all_half) {
            pipeline(std::true_type{});
        } else
        for (uint32_t nt = 0; nt < tn; nt++) {
            const uint4 v0 = sb[(4u * nt) * 64u + l], v1 = sb[(4u * nt + 1u) * 64u + l];
            const ifa_v8i B0 = {(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, 0, 0, 0, 0};
            const ifa_v8i B1 = {(int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w, 0, 0, 0, 0};
            ifa_v8i B2 = {}, B3 = {};
            const uint32_t meta = __builtin_amdgcn_readfirstlane(sw[nt]);
            const bool two = NW == 2 && (meta & 0xffu) == 2u;
            // half-step tile: the first K step alone (the windows' first
            // 16 - shift bases)
            const bool half = (meta >> 8) != 0u;
            if (two) {
                const uint4 v2 = sb[(4u * nt + 2u) * 64u + l], v3 = sb[(4u * nt + 3u) * 64u + l];
                B2 = ifa_v8i{(int)v2.x, (int)v2.y, (int)v2.z, (int)v2.w, 0, 0, 0, 0};
                B3 = ifa_v8i{(int)v3.x, (int)v3.y, (int)v3.z, (int)v3.w, 0, 0, 0, 0};
            }
            const float need = st[32u * nt + g];
            float mx = -1e30f;
#pragma unroll
            for (int p = 0; p < 2; p++) {
                ifa_v16f d0 = mfma_fp4(A[0][2 * p][0], B0, zero);
                ifa_v16f d1 = mfma_fp4(A[0][2 * p + 1][0], B0, zero);
                if (!half) {
                    d0 = mfma_fp4(A[0][2 * p][1], B1, d0);
                    d1 = mfma_fp4(A[0][2 * p + 1][1], B1, d1);
                }
                if (two) {
                    d0 = mfma_fp4(A[NW - 1][2 * p][0], B2, d0);
                    d1 = mfma_fp4(A[NW - 1][2 * p + 1][0], B2, d1);
                    d0 = mfma_fp4(A[NW - 1][2 * p][1], B3, d0);
                    d1 = mfma_fp4(A[NW - 1][2 * p + 1][1], B3, d1);
                }
#pragma unroll
                for (int i = 0; i < 16; i++) mx = fmaxf(fmaxf(d0[i], d1[i]), mx);
            }
            const uint64_t m = __ballot(mx >= need);
#pragma unroll
            for (uint32_t q = 0; q < 4; q++)
                if (m & (0x000000ff000000ffull << (8u * q))) pending |= 1u << (4u * nt + q);
        }
        if (pending && l == 0u) {
            const unsigned int idx = atomicAdd(a.work_count, 1u);
            if (idx < a.work_cap) {
                WorkItem it;
                it.wave = wave;
                it.qb = qb;
                it.pending = pending;
                it.pad = 0;
                a.work[idx] = it;
            }
        }
        // the next iteration rewrites this wave's words: all reads done first
        __builtin_amdgcn_wave_barrier();
    }
}

// LDS bytes of the three-class matrix filter for `tiles` column tiles.
static uint32_t mq3_lds_bytes(uint32_t tiles, uint32_t wg, int nw)
{
    return tiles * (256u * 16u + 32u * 4u) + 8u * 4u + 256u * 4u +
           (wg / 64u) * 3u * m3_blocks(nw) * 4u;
}

// ---------------------------------------------------------------------------
// Dense strands on the matrix cores.
//
// For a query strand of L <= 32 bases the three-class contraction over its
// whole length is the exact match count of every window: with need = L - k -
// nA (nA = A bases of the strand), a window is a hit iff its value D reaches
// need, and its mismatches are m = k - (D - need). So on a clean wave -- no N
// and no piece end in the words its windows read, every window owned and
// inside the chunk and the scanned range, all in one piece -- the dense
// strands [dm_first, n_qs) (all of L <= 32, chosen by the host for their low
// random-window hit rate) are counted here, with the filter's staging and
// operand layout. A workgroup holds a batch of kDmTiles column tiles (four
// strands each) in LDS, and each wave stages its stream once for all of them.
// Hits are listed per accumulator register, in blocks of kDmBlock registers:
// the block's ballots (lanes whose value reaches need) come first, then, after
// a flush if the block's hits could overflow the wave's LDS list, each
// register with hits is listed, the hitting lanes taking slots total + mbcnt.
// Only the flush at a block's start and the one at the wave's end are
// inlined, so the loop stays small. The list is hashed (or written out as
// records) with every lane busy, into LDS copies of the per-strand sums that
// go to the query's accumulators when the workgroup ends. The VALU dense
// kernels take those strands only on waves that are not clean.
//
// Grid: x = workgroups walking waves (XCD-aware), y = batch of column tiles.
// ---------------------------------------------------------------------------

constexpr uint32_t kDmTiles = 4;     // column tiles per batch (16 strands)
constexpr uint32_t kDmBlock = 8;     // accumulator registers listed per block
constexpr uint32_t kDmList = 64u * kDmBlock;   // hit-list entries per wave
constexpr uint32_t kDmReps = 8;      // copies of each strand's sums in LDS
// the per-strand LDS arrays below hold 32 strands
static_assert(4u * kDmTiles <= 32u, "dense matrix batch too large");

// Is the 1024-window wave whose window starts begin at word w0 clean (see
// above) for strands of at most 32 bases? Windows start in words w0 ..
// w0 + 31 and read up to word w0 + 32. Called by all 64 lanes.
__device__ __forceinline__ bool wave_is_clean(const ScanArgs &a, uint32_t w0)
{
    const uint32_t l = threadIdx.x & 63u;
    if (w0 + 32u > a.w_end || 32ull * w0 < (uint64_t)a.own_from ||
        32ull * (w0 + 33u) > a.chunk_len)
        return false;
    uint32_t bad = 0;
    if (l <= 32u) bad = a.nm[w0 + l] | a.em[w0 + l];
    return !__any(bad != 0u);
}

// LDS state of a dense matrix workgroup (one batch of kDmTiles column tiles).
struct DmShared {
    const uint32_t *kq;             // [32] k | strand << 16 per strand of the batch
    const uint32_t *qid;            // [32] caller's query index per strand
    uint32_t *cnt;                  // [32][kDmReps] hit counts
    unsigned long long *dig;        // [32][kDmReps] digests
};

// Hash (or write out as records) the `total` hits listed in a wave's list,
// with every lane. An entry is (D - need) | lane << 8 | register << 14 | row
// tile << 18 | tile << 21: the lane that held the value gives its column
// (strand 4 tile + column / 8 of the batch, shift column % 8), and the
// mismatches are k - (D - need). (D and need may be negative: D counts an A
// of the query as -1 where the reference base is not A; D - need of a hit is
// in [0, k].) Counts and digests go to one of kDmReps copies of the
// strand's sums (by lane), so that lanes hashing hits of one strand do not
// queue on one LDS address. Called by all 64 lanes of the wave.
__device__ __forceinline__ void dm_flush(const ScanArgs &a, const uint32_t *list, uint32_t total,
                                         uint32_t contig, uint32_t pos0, const DmShared &sh)
{
    const uint32_t l = threadIdx.x & 63u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    unsigned long long base = 0;
    if (a.sink == kSinkRecords) {
        if (l == 0u) base = atomicAdd(a.hit_count, (unsigned long long)total);
        base = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    }
    for (uint32_t e = l; e < total; e += 64u) {
        const uint32_t ent = list[e];
        const uint32_t el = (ent >> 8) & 63u, i = (ent >> 14) & 15u;
        const uint32_t u = (ent >> 18) & 7u, nt = ent >> 21;
        const uint32_t col = el & 31u, eh = el >> 5;
        const uint32_t qb = 4u * nt + (col >> 3);            // strand in the batch
        const uint32_t kq = sh.kq[qb];
        // window of register i: row tile u, group 8 (i / 4) + 4 h + i % 4
        const uint32_t win = 256u * u + 8u * (8u * (i >> 2) + 4u * eh + (i & 3u)) + (col & 7u);
        const uint32_t m = (kq & 0xffffu) - (ent & 0xffu);
        if (a.sink == kSinkRecords) {
            if (base + e < a.hit_cap)
                a.hits[base + e] = make_uint4(sh.qid[qb], contig, pos0 + win, (kq >> 16) | (m << 16));
        } else {
            const uint32_t rep = kDmReps * qb + (l & (kDmReps - 1u));
            atomicAdd(&sh.cnt[rep], 1u);
            atomicAdd(&sh.dig[rep], (unsigned long long)hit_hash(contig, pos0 + win, kq >> 16, m, 0u));
        }
    }
    // the list is rewritten next: every read is done first
    __builtin_amdgcn_wave_barrier();
}

template <int WG>
__global__ __launch_bounds__(WG) void scan_dense_mfma3_kernel(ScanArgs a)
{
    constexpr uint32_t kBlocks = m3_blocks(1), kWords = 3 * kBlocks;
    extern __shared__ uint4 lds[];
    const uint32_t n_dm = a.n_qs - a.dm_first;                      // strands on the matrix cores
    const uint32_t n_tiles = (n_dm + 3u) / 4u;
    const uint32_t t0 = kDmTiles * blockIdx.y;                      // first tile of the batch
    const uint32_t tn = min(n_tiles, t0 + kDmTiles) - t0;
    const uint32_t nq = min(4u * tn, n_dm - 4u * t0);               // strands of the batch
    uint4 *sb = lds;                                                // [tile][2 K steps][64]
    float *st = reinterpret_cast<float *>(lds + 128u * kDmTiles);   // [tile][32] need
    unsigned long long *sdig =
        reinterpret_cast<unsigned long long *>(st + 32u * kDmTiles); // [32][kDmReps]
    uint32_t *scnt = reinterpret_cast<uint32_t *>(sdig + 32u * kDmReps); // [32][kDmReps]
    uint32_t *skq = scnt + 32u * kDmReps;                           // [32]
    uint32_t *sqid = skq + 32u;                                     // [32]
    uint32_t *sp = sqid + 32u;                                      // [256]
    const uint32_t wid = threadIdx.x >> 6;
    uint32_t *flat = sp + 256u + wid * (kWords + kDmList);          // this wave's words
    uint32_t *list = flat + kWords;                                 // this wave's hit list
    for (uint32_t i = threadIdx.x; i < 128u * tn; i += WG) sb[i] = a.dm_b[128u * t0 + i];
    for (uint32_t i = threadIdx.x; i < 32u * tn; i += WG) st[i] = a.dm_t[32u * t0 + i];
    for (uint32_t i = threadIdx.x; i < 32u * kDmReps; i += WG) {
        sdig[i] = 0ull;
        scnt[i] = 0u;
    }
    for (uint32_t i = threadIdx.x; i < nq; i += WG) {
        const QS d = load_qs(a, a.dm_first + 4u * t0 + i);
        skq[i] = d.k | (d.strand << 16);
        sqid[i] = d.qid;
    }
    for (uint32_t i = threadIdx.x; i < 256u; i += WG) sp[i] = kSpread.v[i];
    __syncthreads();
    const DmShared sh{skq, sqid, scnt, sdig};

    const uint32_t l = threadIdx.x & 63u;
    const uint32_t g = l & 31u, h = l >> 5;
    const uint32_t last = (uint32_t)((a.chunk_len + 31) >> 5) + kPadWords - 1;
    const uint32_t n_waves = (a.w_end - a.w_begin + 31u) >> 5;
    const uint32_t stride = gridDim.x * (WG / 64u);
    const ifa_v16f zero = {};
    // piece of the last wave walked: waves come in increasing order, so the
    // next wave's piece is found by stepping forward from it
    uint32_t pidx = 0xffffffffu;
    for (uint32_t wave = xcd_local_x() * (WG / 64u) + wid; wave < n_waves; wave += stride) {
        const uint32_t w0 = a.w_begin + 32u * wave;
        if (!wave_is_clean(a, w0)) continue;
        // contig and position of the wave's first window (one piece)
        uint32_t contig = 0, pos0 = 0;
        {
            const uint64_t first = 32ull * w0;
            if (pidx == 0xffffffffu) {
                pidx = find_piece(a, first);
            } else {
                while (pidx + 1u < a.n_pieces && a.pieces[pidx + 1u].start <= first) pidx++;
            }
            const Piece pc = a.pieces[pidx];
            contig = pc.contig;
            pos0 = (uint32_t)(pc.contig_off + (first - pc.start));
        }
        // stage the indicator words of blocks 4j .. 4j + 3 (lane j)
        if (l < kBlocks / 4u) {
            const uint32_t w = min(w0 + l, last);
            const uint32_t ch = a.hi[w], cl = a.lo[w];
            const uint32_t m = 0x22222222u;
            uint32_t v[12];
#pragma unroll
            for (uint32_t q = 0; q < 4; q++) {
                const uint32_t s1 = sp[(ch >> (8u * q)) & 0xffu];
                const uint32_t s0 = sp[(cl >> (8u * q)) & 0xffu];
                v[3 * q] = ~s1 & s0 & m;           // C (hi 0, lo 1)
                v[3 * q + 1] = s1 & s0 & m;        // G (1, 1)
                v[3 * q + 2] = s1 & ~s0 & m;       // T (1, 0)
            }
            uint4 *dst = reinterpret_cast<uint4 *>(flat + 12u * l);
            dst[0] = make_uint4(v[0], v[1], v[2], v[3]);
            dst[1] = make_uint4(v[4], v[5], v[6], v[7]);
            dst[2] = make_uint4(v[8], v[9], v[10], v[11]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        ifa_v8i A[4][2];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t *f = flat + 3u * (32u * u + g) + 4u * h;
#pragma unroll
            for (int t = 0; t < 2; t++)
                A[u][t] = ifa_v8i{(int)f[8 * t], (int)f[8 * t + 1], (int)f[8 * t + 2],
                                  (int)f[8 * t + 3], 0, 0, 0, 0};
        }
        uint32_t total = 0;   // wave-uniform: entries in the list
        for (uint32_t nt = 0; nt < tn; nt++) {
            const uint4 v0 = sb[(2u * nt) * 64u + l], v1 = sb[(2u * nt + 1u) * 64u + l];
            const ifa_v8i B0 = {(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, 0, 0, 0, 0};
            const ifa_v8i B1 = {(int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w, 0, 0, 0, 0};
            // columns past the last strand never hit (their need is huge)
            const float need = st[32u * nt + g];
            const uint32_t lane_ent = (l << 8) | (nt << 21);
#pragma unroll
            for (int p = 0; p < 2; p++) {
                ifa_v16f d0 = mfma_fp4(A[2 * p][0], B0, zero);
                ifa_v16f d1 = mfma_fp4(A[2 * p + 1][0], B0, zero);
                d0 = mfma_fp4(A[2 * p][1], B1, d0);
                d1 = mfma_fp4(A[2 * p + 1][1], B1, d1);
                // blocks of kDmBlock registers: all their ballots first, then
                // (after a flush if the list could overflow) the listing
#pragma unroll
                for (int b = 0; b < 32 / (int)kDmBlock; b++) {
                    uint64_t mb[kDmBlock];
                    uint32_t sum = 0;
#pragma unroll
                    for (int j = 0; j < (int)kDmBlock; j++) {
                        const int r = (int)kDmBlock * b + j;
                        mb[j] = __ballot((r < 16 ? d0[r & 15] : d1[r & 15]) >= need);
                        sum += (uint32_t)__popcll(mb[j]);
                    }
                    if (sum == 0u) continue;
                    if (total + sum > kDmList) {
                        dm_flush(a, list, total, contig, pos0, sh);
                        total = 0;
                    }
#pragma unroll
                    for (int j = 0; j < (int)kDmBlock; j++) {
                        const int r = (int)kDmBlock * b + j;
                        const float v = r < 16 ? d0[r & 15] : d1[r & 15];
                        if (mb[j] == 0u) continue;
                        if (v >= need) {
                            const uint32_t slot = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(mb[j] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb[j], total));
                            list[slot] = __builtin_amdgcn_cvt_pk_u8_f32(
                                v - need, 0u,
                                lane_ent | ((uint32_t)(r & 15) << 14) | ((uint32_t)(2 * p + (r >> 4)) << 18));
                        }
                        total += (uint32_t)__popcll(mb[j]);
                    }
                }
            }
        }
        if (total) dm_flush(a, list, total, contig, pos0, sh);
        // the next wave rewrites this wave's words: all reads done first
        __builtin_amdgcn_wave_barrier();
    }
    if (a.sink == kSinkCountDigest) {
        __syncthreads();
        // one addition per strand of the batch to its query's accumulators
        for (uint32_t i = threadIdx.x; i < nq; i += WG) {
            uint32_t c = 0;
            unsigned long long s = 0;
#pragma unroll
            for (uint32_t j = 0; j < kDmReps; j++) {
                c += scnt[kDmReps * i + j];
                s += sdig[kDmReps * i + j];
            }
            if (c == 0u) continue;
            const uint32_t slot = sqid[i] * kStripes + blockIdx.x % kStripes;
            atomicAdd(&a.q_count[slot], (unsigned long long)c);
            atomicAdd(&a.q_digest[slot], s);
        }
    }
}

// LDS bytes of the dense matrix kernel (one batch of kDmTiles column tiles).
static uint32_t dm3_lds_bytes(uint32_t wg)
{
    return kDmTiles * (128u * 16u + 32u * 4u) + 32u * kDmReps * (8u + 4u) + 2u * 32u * 4u +
           256u * 4u + (wg / 64u) * (3u * m3_blocks(1) + kDmList) * 4u;
}

// One wave per work item (grid-stride). Does nothing when the filter kernel
// overflowed the list: the host then grows it and runs the sparse part again.
template <int W>
__global__ __launch_bounds__(256) void scan_resolve_kernel(ScanArgs a)
{
    const unsigned int count = *a.work_count;
    if (count > a.work_cap) return;
    const uint32_t waves = gridDim.x * 4u;
    const uint32_t slot = blockIdx.x * 4u + (threadIdx.x >> 6);
    const IFA_CONST uint32_t *work = as_const(reinterpret_cast<const uint32_t *>(a.work));
    for (uint32_t i = slot; i < count; i += waves) {
        const uint32_t wave = work[4u * i], qb = work[4u * i + 1];
        uint32_t pending = work[4u * i + 2];
        Lane ln = make_lane<W>(a, wave * 64u + (threadIdx.x & 63u));
        while (pending) {
            const uint32_t j = __builtin_ctz(pending);
            pending &= pending - 1u;
            const QS d = load_qs(a, qb + j);
            resolve<W>(a, d, ln, filter_cand_words<W>(a, d, ln, strand_filter_words(a, qb + j)),
                       wave);
        }
    }
}

// Dense query strands [n_sparse, n_qs): strands whose filter would pass a
// window in 1/32 of the waves or more (short queries with high k, long
// queries with k >= 16). Each lane counts its W windows' mismatches word by word, all
// windows at once; after each 32-base word the wave stops with this strand
// once no window of any lane is still within k (the paper's early exit, per
// word). Windows within k after the last word are hits; plain lanes emit them
// here. Other lanes (N, piece end, carried prefix, chunk tail) are left to
// scan_dense_cold_kernel, so that their code does not weigh on this loop's
// registers. Dense strands come sorted by L descending (those counted on the
// matrix cores last, again by L descending), so the cached word-0 slices can
// be masked in place and are rebuilt once at that seam.
// Count+digest in the dense kernel: list the hits in LDS and hash them with
// every lane busy (W = 16); at W = 32 the list would halve the occupancy.
template <int W>
constexpr bool kCompactHits = W <= 16;

template <int W>
__device__ __forceinline__ void dense_strand(const ScanArgs &a, const QS &d, const Lane &ln,
                                             bool plain, uint32_t contig, uint32_t pos0,
                                             const uint32_t (&sh)[W], const uint32_t (&sl)[W],
                                             uint32_t &cnt, uint64_t &dig, uint32_t *hits,
                                             const uint32_t *lane_pos)
{
    uint32_t m[W];
    uint32_t mn = 0xffffffffu;
#pragma unroll
    for (int b = 0; b < W; b++) {
        uint32_t diff = __builtin_amdgcn_bitop3_b32(sh[b], d.qh, d.qn, IFA_XOR_OR);
        diff = __builtin_amdgcn_bitop3_b32(diff, sl[b], d.ql, IFA_OR_XOR);
        m[b] = __popc(diff);
        mn = min(mn, m[b]);
    }
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    uint32_t hp = ln.h1, lp = ln.l1;
    for (uint32_t t = 1; t < d.nw; t++) {
        if (!__any(plain && mn <= d.k)) break;
        const uint32_t x = ln.w + t + 1;
        const uint32_t hn = a.hi[x], lnw = a.lo[x];
        const uint32_t qh = qw[3 * t], ql = qw[3 * t + 1], qn = qw[3 * t + 2];
        const uint32_t lmask = low_mask(d.len - 32u * t);
        mn = 0xffffffffu;
#pragma unroll
        for (int b = 0; b < W; b++) {
            const uint32_t s = ln.off + (uint32_t)b;
            uint32_t diff = __builtin_amdgcn_bitop3_b32(funnel(hn, hp, s), qh, qn, IFA_XOR_OR);
            diff = __builtin_amdgcn_bitop3_b32(diff, funnel(lnw, lp, s), ql, IFA_OR_XOR);
            m[b] += __popc(diff & lmask);
            mn = min(mn, m[b]);
        }
        hp = hn;
        lp = lnw;
    }
    if (!__any(plain && mn <= d.k)) return;
    if constexpr (!kCompactHits<W>) {
        // 32 windows per lane: count, emit and hash in place (a hit mask and
        // list would cost a quarter of the occupancy)
        if (plain && mn <= d.k) {
            uint32_t c = 0;
#pragma unroll
            for (int b = 0; b < W; b++) c += m[b] <= d.k ? 1u : 0u;
            cnt += c;
            if (a.sink == kSinkRecords) {
                unsigned long long slot = atomicAdd(a.hit_count, (unsigned long long)c);
#pragma unroll
                for (int b = 0; b < W; b++) {
                    if (m[b] <= d.k) {
                        write_record(a, slot, d, contig, pos0 + b, m[b], 0u);
                        slot++;
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < W; b++)
                    if (m[b] <= d.k) dig += hit_hash(contig, pos0 + b, d.strand, m[b], 0u);
            }
        }
        return;
    }
    const bool live = plain && mn <= d.k;
    if (a.sink == kSinkRecords) {
        // the lane's hits: bit b for window b
        uint32_t hm = 0;
        if (live) {
#pragma unroll
            for (int b = 0; b < W; b++) hm |= (m[b] <= d.k ? 1u : 0u) << b;
        }
        const uint32_t c = __popc(hm);
        cnt += c;
        if (hm) {
            unsigned long long slot = atomicAdd(a.hit_count, (unsigned long long)c);
#pragma unroll
            for (int b = 0; b < W; b++) {
                if ((hm >> b) & 1u) {
                    write_record(a, slot, d, contig, pos0 + b, m[b], 0u);
                    slot++;
                }
            }
        }
    } else {
        // Hash the hits with every lane busy: they are listed in this wave's
        // LDS area window by window (the lanes hitting window b, from one
        // ballot, take the slots after the hits of windows < b), then lane i
        // hashes entries i, i + 64, ... Hashing in place would run the hash
        // for all 64 lanes at every window any lane hits. An entry is
        // m | lane << 16 | b << 24; the lane's contig and first position sit
        // in LDS. The wave's hit total goes to lane 0's count (the query's
        // count is a wave sum).
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t lane16 = lane << 16;
        // one signed compare per window: lanes without a hit compare with -1
        const int kk = live ? (int)d.k : -1;
        uint32_t total = 0;   // wave-uniform
#pragma unroll
        for (int b = 0; b < W; b++) {
            const bool hit = (int)m[b] <= kk;
            const uint64_t mb = __ballot(hit);
            if (mb == 0u) continue;
            if (hit) {
                const uint32_t slot = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, total));
                hits[slot] = m[b] | lane16 | ((uint32_t)b << 24);
            }
            total += (uint32_t)__popcll(mb);
        }
        if (lane == 0u) cnt += total;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t i = lane; i < total; i += 64u) {
            const uint32_t e = hits[i], hl = (e >> 16) & 0xffu;
            dig += hit_hash(lane_pos[2u * hl], lane_pos[2u * hl + 1u] + (e >> 24), d.strand,
                            e & 0xffffu, 0u);
        }
        // the next strand rewrites the list: every read is done first
        __builtin_amdgcn_wave_barrier();
    }
}

template <int W>
__global__ __launch_bounds__(256) void scan_dense_kernel(ScanArgs a)
{
    // per wave: the hit list of the strand being hashed (at most 64 W hits)
    // and the contig and first position of every lane
    __shared__ uint32_t hit_lds[4][kCompactHits<W> ? 64 * W : 1];
    __shared__ uint32_t pos_lds[4][kCompactHits<W> ? 2 * 64 : 1];
    const uint32_t gl = blockIdx.x * 256u + threadIdx.x;
    const Lane ln = make_lane<W>(a, gl);
    const uint32_t wave = gl >> 6;
    // the launch for the matrix-counted strands takes only the waves the
    // matrix kernel leaves out
    if (a.dense_unclean && wave_is_clean(a, a.w_begin + 32u * wave)) return;
    uint32_t *hits = hit_lds[threadIdx.x >> 6];
    uint32_t *lane_pos = pos_lds[threadIdx.x >> 6];
    uint32_t sh[W], sl[W];
#pragma unroll
    for (int b = 0; b < W; b++) {
        sh[b] = funnel(ln.h1, ln.h0, ln.off + (uint32_t)b);
        sl[b] = funnel(ln.l1, ln.l0, ln.off + (uint32_t)b);
    }
    // plain lanes find their contig and position once for every strand
    const bool plain = ln.active && lane_is_plain(a, ln);
    uint32_t contig = 0, pos0 = 0;
    if (plain) {
        const uint64_t first = 32ull * ln.w + ln.off;
        const Piece pc = a.pieces[find_piece(a, first)];
        contig = pc.contig;
        pos0 = (uint32_t)(pc.contig_off + (first - pc.start));
    }
    if (kCompactHits<W>) {
        lane_pos[2u * (threadIdx.x & 63u)] = contig;
        lane_pos[2u * (threadIdx.x & 63u) + 1u] = pos0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    uint32_t cur_len = 32;
    // strands [dense_begin, dense_end): with strands counted on the matrix
    // cores, the others in one launch and those in a second one (waves the
    // matrix kernel leaves out), each range by L descending
    const uint32_t q_end = a.dense_end;
    // both strands of a query are adjacent: their counts are summed before
    // the wave-wide reduction
    uint32_t cnt = 0, qid = 0xffffffffu;
    uint64_t dig = 0;
    // the next strand's descriptor is loaded while this one runs
    QS nxt = load_qs(a, a.dense_begin);
    for (uint32_t q = a.dense_begin; q < q_end; q++) {
        const QS d = nxt;
        if (q + 1u < q_end) nxt = load_qs(a, q + 1u);
        if (d.qid != qid) {
            if (a.sink == kSinkCountDigest && qid != 0xffffffffu)
                wave_add_stats(a, qid, cnt, dig, wave);
            cnt = 0;
            dig = 0;
            qid = d.qid;
        }
        if (d.len < cur_len) {
            mask_slices<W>(sh, sl, d.len);
            cur_len = d.len;
        }
        // keep the hash keys of the W windows from being hoisted out of the
        // strand loop (32 more live registers, half the occupancy)
        asm volatile("" : "+v"(contig), "+v"(pos0));
        dense_strand<W>(a, d, ln, plain, contig, pos0, sh, sl, cnt, dig, hits, lane_pos);
    }
    if (a.sink == kSinkCountDigest && qid != 0xffffffffu) wave_add_stats(a, qid, cnt, dig, wave);
}

// Dense query strands on the lanes scan_dense_kernel leaves out (an N, a
// piece end, the carried prefix or the chunk tail among their bases): the
// exact serial test. Waves without such a lane return at once. Such lanes are
// few and scattered (one to a few per wave), so the wave's lanes take the
// strands (lane j: strands n_sparse + j, + 64, ...) and each tests its strand
// against the windows of every cold lane of the wave in turn, whose words are
// broadcast; count+digest sums go to the query's stripe once per strand.
template <int W>
__global__ __launch_bounds__(256) void scan_dense_cold_kernel(ScanArgs a)
{
    const uint32_t gl = blockIdx.x * 256u + threadIdx.x;
    const Lane ln = make_lane<W>(a, gl);
    const uint64_t cold = __ballot(ln.active && !lane_is_plain(a, ln));
    if (cold == 0u) return;
    const uint32_t l = threadIdx.x & 63u;
    const uint32_t wave = gl >> 6;
    const uint32_t q_end =
        a.dm_first < a.n_qs && wave_is_clean(a, a.w_begin + 32u * wave) ? a.dm_first : a.n_qs;
    for (uint32_t q0 = a.n_sparse; q0 < q_end; q0 += 64u) {
        const bool on = q0 + l < q_end;
        const QS d = load_qs(a, on ? q0 + l : q0);
        uint32_t cnt = 0;
        uint64_t dig = 0;
        for (uint64_t rest = cold; rest != 0u; rest &= rest - 1u) {
            const int c = (int)__builtin_ctzll(rest);
            Lane lc;
            lc.w = (uint32_t)__builtin_amdgcn_readlane((int)ln.w, c);
            lc.off = (uint32_t)__builtin_amdgcn_readlane((int)ln.off, c);
            lc.h0 = (uint32_t)__builtin_amdgcn_readlane((int)ln.h0, c);
            lc.h1 = (uint32_t)__builtin_amdgcn_readlane((int)ln.h1, c);
            lc.l0 = (uint32_t)__builtin_amdgcn_readlane((int)ln.l0, c);
            lc.l1 = (uint32_t)__builtin_amdgcn_readlane((int)ln.l1, c);
            lc.n0 = (uint32_t)__builtin_amdgcn_readlane((int)ln.n0, c);
            lc.n1 = (uint32_t)__builtin_amdgcn_readlane((int)ln.n1, c);
            lc.active = true;
            lc.plain = 0;
            if (on && filter_cand_words<W>(a, d, lc, 1u)) exact_serial<W>(a, d, lc, cnt, dig);
        }
        if (a.sink == kSinkCountDigest && on && cnt != 0u) {
            const uint32_t slot = d.qid * kStripes + wave % kStripes;
            atomicAdd(&a.q_count[slot], (unsigned long long)cnt);
            atomicAdd(&a.q_digest[slot], (unsigned long long)dig);
        }
    }
}

// Windows that hang off a contig end (soft clip at contig boundaries). For a
// query strand with clip limit C = min(maxN, L - 1) a piece has 2C window
// slots: slot i < C is the start i - C (a piece holding the contig's first
// base), slot C + o - 1 the start n - L + o, o in [1, C] (a piece holding its
// last base; starts below 0 are left slots). Bases off the contig read as N
// and at most C of them may be in a window. A window belongs to the piece
// (and chunk) owning its last on-contig base and to the word range holding
// that base, so each is tested once; all of its on-contig bases lie in that
// piece, because a contig's first piece starts at its first base and a chunk
// repeats the kCarry bases before a split.
//
// Task (b, q): one wave tests strand q against pieces [b P, b P + P), P =
// 64 / 2C pieces side by side (one piece over several rounds when 2C > 64).
// Tasks are walked grid-stride with (b, q) stepped incrementally, 32-bit.
// Coordinates are piece-local (contigs and chunks are below 2^31 bases).
__global__ __launch_bounds__(256) void scan_edge_kernel(ScanArgs a)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t waves = gridDim.x * 4u;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t nb = (a.n_pieces + a.edge_pmin - 1u) / a.edge_pmin;
    const uint32_t dq = waves % a.n_qs, db = waves / a.n_qs;
    uint32_t q = wave % a.n_qs, b = wave / a.n_qs;
    const uint32_t own_from = (uint32_t)a.own_from;
    const IFA_CONST uint32_t *pw = as_const(reinterpret_cast<const uint32_t *>(a.pieces));
    // task t = b n_qs + q advances by `waves`: (b, q) += (db, dq) with a carry
    for (; b < nb; q += dq, b += db + (q >= a.n_qs ? 1u : 0u), q -= (q >= a.n_qs ? a.n_qs : 0u)) {
        const QS d = load_qs(a, q);
        const int32_t L = (int32_t)d.len;
        const int32_t C = (int32_t)d.maxn < L - 1 ? (int32_t)d.maxn : L - 1;
        if (C <= 0) continue;
        const uint32_t S = 2u * (uint32_t)C;               // slots per piece
        const uint32_t P = S <= 64u ? 64u / S : 1u;         // pieces per wave
        if (b * P >= a.n_pieces) continue;
        const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
        uint32_t cnt = 0;
        uint64_t dig = 0;
        for (uint32_t s0 = 0; s0 < P * S; s0 += 64u) {
            const uint32_t slot = s0 + lane;
            const uint32_t pi = b * P + slot / S;
            const int32_t i = (int32_t)(slot % S);
            bool ok = slot < P * S && pi < a.n_pieces;
            uint32_t start = 0, len = 0, flags = 0, contig = 0;
            int32_t c0 = 0;
            if (ok) {
                const IFA_CONST uint32_t *r = pw + 8u * pi;   // Piece, 8 words
                start = r[0];
                len = r[2];
                c0 = (int32_t)r[4];
                contig = r[6];
                flags = r[7];
            }
            const bool has_end = (flags & kPieceContigEnd) != 0u;
            // window start pl and its on-contig bases [f, e], piece-local
            int32_t pl, f, e, off;
            if (i < C) {
                ok = ok && (flags & kPieceContigStart) != 0u;   // then c0 == 0
                pl = i - C;
                f = 0;
                e = (has_end && pl > (int32_t)len - L) ? (int32_t)len - 1 : pl + L - 1;
                off = L - (e + 1);
            } else {
                const int32_t o = i - C + 1;
                pl = (int32_t)len - L + o;
                ok = ok && has_end && c0 + pl >= 0 && pl >= 0;
                f = pl;
                e = (int32_t)len - 1;
                off = o;
            }
            const int32_t own_lo = own_from > start ? (int32_t)(own_from - start) : 0;
            ok = ok && off <= C && e >= own_lo && e <= (int32_t)len - 1 && f <= e;
            if (ok) {
                const uint32_t ew = (start + (uint32_t)e) >> 5;
                ok = ew >= a.w_begin && ew < a.w_end;
            }
            uint32_t m = 0, nref = 0;
            if (ok) {
                for (uint32_t t = 0; t < d.nw; t++) {
                    const int32_t cw = pl + 32 * (int32_t)t;   // piece-local base of bit 0
                    const uint32_t lmask = low_mask((uint32_t)(L - 32 * (int32_t)t));
                    const int32_t lo_b = min(max(f - cw, 0), 32);
                    const int32_t hi_b = min(max(e + 1 - cw, 0), 32);
                    uint32_t rh = 0u, rl = 0u, rn = 0u, vm = 0u;
                    if (lo_b < hi_b) {
                        const uint32_t u = start + (uint32_t)(cw + lo_b);   // on-contig base
                        const uint32_t x = u >> 5, sh = u & 31u;
                        rh = funnel(a.hi[x + 1], a.hi[x], sh) << lo_b;
                        rl = funnel(a.lo[x + 1], a.lo[x], sh) << lo_b;
                        rn = funnel(a.nm[x + 1], a.nm[x], sh) << lo_b;
                        vm = low_mask((uint32_t)hi_b) & ~low_mask((uint32_t)lo_b);
                    }
                    const uint32_t rne = ((rn & vm) | ~vm) & lmask;   // N or off the contig
                    const uint32_t diff =
                        (qw[3 * t] ^ rh) | (qw[3 * t + 1] ^ rl) | qw[3 * t + 2];
                    if (a.policy == kNSeparate)
                        m += __popc(diff & ~rne & lmask);
                    else
                        m += __popc((diff | rne) & lmask);
                    nref += __popc(rne);
                }
                ok = m <= d.k && (a.policy != kNSeparate || nref <= d.maxn);
            }
            if (ok) {
                const uint32_t pos = (uint32_t)(c0 + pl);
                if (a.sink == kSinkRecords) {
                    write_record(a, atomicAdd(a.hit_count, 1ull), d, contig, pos, m, nref);
                } else {
                    cnt += 1;
                    dig += hit_hash(contig, pos, d.strand, m, nref);
                }
            }
        }
        if (a.sink == kSinkCountDigest) wave_add_stats(a, d.qid, cnt, dig, wave);
    }
}

// ---------------------------------------------------------------------------
// indexed mode
// ---------------------------------------------------------------------------

// Bits [lo, lo + mask) squeezed out of x (the masked centre of a seed).
__device__ __forceinline__ uint32_t squeeze_mask(uint32_t x, uint32_t lo, uint32_t mask)
{
    return (x & low_mask(lo)) | ((x >> (lo + mask)) << lo);
}

// Equality bits of query word t of strand d against the window at chunk
// position 32 w + b: 1 where both bases are A/C/G/T and equal (0 past L).
__device__ __forceinline__ uint32_t eq_word(const ScanArgs &a, const QS &d,
                                            const IFA_CONST uint32_t *qw, uint32_t w, uint32_t b,
                                            uint32_t t)
{
    if (t >= d.nw) return 0u;
    const uint32_t x = w + t;
    const uint32_t rh = funnel(a.hi[x + 1], a.hi[x], b);
    const uint32_t rl = funnel(a.lo[x + 1], a.lo[x], b);
    const uint32_t rn = funnel(a.nm[x + 1], a.nm[x], b);
    const uint32_t diff = (qw[3 * t] ^ rh) | (qw[3 * t + 1] ^ rl) | qw[3 * t + 2] | rn;
    return ~diff & low_mask(d.len - 32u * t);
}

// A seed of strand q at offset i matched the reference at chunk position r:
// test window p = r - i. It is reported when it is a hit (every query word,
// the N rule, piece ends, chunk ownership), holds at least the strand's
// threshold of error-free seeds, and i is its first error-free seed, so that
// each window is reported by exactly one of its seeds.
__device__ void seed_verify(const ScanArgs &a, uint32_t q, uint32_t i, uint64_t r, uint32_t stripe)
{
    if (r < i) return;
    const uint64_t p = r - i;
    const QS d = load_qs(a, q);
    const uint32_t L = d.len;
    if (p + L > a.chunk_len || p + L - 1 < (uint64_t)a.own_from) return;
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    const uint32_t w = (uint32_t)(p >> 5), b = (uint32_t)(p & 31u);
    uint32_t m = 0, nref = 0, ends = 0;
    for (uint32_t t = 0; t < d.nw; t++) {
        const uint32_t i0 = 32u * t;
        const uint32_t lmask = low_mask(L - i0);
        const uint32_t emask = (L - 1 > i0) ? low_mask(L - 1 - i0) : 0u;
        const uint32_t x = w + t;
        const uint32_t rh = funnel(a.hi[x + 1], a.hi[x], b);
        const uint32_t rl = funnel(a.lo[x + 1], a.lo[x], b);
        const uint32_t rn = funnel(a.nm[x + 1], a.nm[x], b);
        const uint32_t re = funnel(a.em[x + 1], a.em[x], b);
        const uint32_t diff = (qw[3 * t] ^ rh) | (qw[3 * t + 1] ^ rl) | qw[3 * t + 2];
        ends |= re & emask;
        if (a.policy == kNSeparate)
            m += __popc(diff & ~rn & lmask);
        else
            m += __popc((diff | rn) & lmask);
        nref += __popc(rn & lmask);
    }
    if (ends || m > d.k || (a.policy == kNSeparate && nref > d.maxn)) return;
    // error-free seeds, in offset order; a seed spans at most two words
    const SeedInfo *si = a.seed_info + q;
    const uint32_t k = si->k, thr = si->thr;
    const uint32_t lo = (k - a.seed_mask) / 2;
    const uint32_t unm = low_mask(lo) | (low_mask(k) & ~low_mask(lo + a.seed_mask));
    uint32_t cnt = 0;
    uint32_t cur = eq_word(a, d, qw, w, b, 0);
    for (uint32_t t = 0; t < d.nw && cnt < thr; t++) {
        const uint32_t nxt = eq_word(a, d, qw, w, b, t + 1);
        uint32_t v = si->valid[t];
        while (v && cnt < thr) {
            const uint32_t o = __builtin_ctz(v);
            v &= v - 1u;
            if ((funnel(nxt, cur, o) & unm) != unm) continue;
            if (32u * t + o < i) return;   // an earlier seed reports this window
            cnt++;
        }
        cur = nxt;
    }
    if (cnt < thr) return;
    const Piece pc = a.pieces[find_piece(a, p)];
    const uint32_t pos = (uint32_t)(pc.contig_off + (p - pc.start));
    if (a.sink == kSinkRecords) {
        write_record(a, atomicAdd(a.hit_count, 1ull), d, pc.contig, pos, m, nref);
    } else {
        const uint32_t slot = d.qid * kStripes + stripe % kStripes;
        atomicAdd(&a.q_count[slot], 1ull);
        atomicAdd(&a.q_digest[slot], (unsigned long long)hit_hash(pc.contig, pos, d.strand, m, nref));
    }
}

// Indexed mode (Methods, "Algorithm Design"): every lane takes the 32 seed
// starts of a plane word of the range, forms the seed key of each start for
// every seed length of the query set (no key where an unmasked base is N),
// and looks it up in that length's bucketed table of query seeds; each
// matching (strand, offset) entry names one window to verify.
__global__ __launch_bounds__(256) void scan_seed_kernel(ScanArgs a)
{
    const uint32_t lanes = gridDim.x * blockDim.x;
    for (uint32_t w = a.w_begin + blockIdx.x * blockDim.x + threadIdx.x; w < a.w_end; w += lanes) {
        const uint32_t h0 = a.hi[w], h1 = a.hi[w + 1], l0 = a.lo[w], l1 = a.lo[w + 1];
        const uint32_t n0 = a.nm[w], n1 = a.nm[w + 1];
#pragma unroll 1
        for (uint32_t c = 0; c < a.seed_ncfg; c++) {
            const SeedTable tab = a.seed_tab[c];
            const uint32_t k = tab.k, bits = tab.bits;
            const uint32_t lo = (k - a.seed_mask) / 2, u = k - a.seed_mask;
            const uint32_t km = low_mask(k);
            const uint32_t unm = low_mask(lo) | (km & ~low_mask(lo + a.seed_mask));
            const uint32_t *dir = tab.dir;
            const uint2 *ent = tab.ent;
#pragma unroll 1
            for (uint32_t b = 0; b < 32u; b++) {
                const uint64_t r = 32ull * w + b;
                if (r + k > a.chunk_len) break;
                if (funnel(n1, n0, b) & unm) continue;
                const uint32_t key = (squeeze_mask(funnel(h1, h0, b) & km, lo, a.seed_mask) << u) |
                                     squeeze_mask(funnel(l1, l0, b) & km, lo, a.seed_mask);
                const uint32_t bit = seed_bit(key, tab.key_bits);
                if (!((tab.bm[bit >> 5] >> (bit & 31u)) & 1u)) continue;
                const uint32_t bk = (key * 0x9E3779B1u) >> (32u - bits);
                const uint32_t e1 = dir[bk + 1];
                for (uint32_t e = dir[bk]; e < e1; e++) {
                    const uint2 en = ent[e];
                    if (en.x == key) seed_verify(a, en.y >> 8, en.y & 255u, r, w);
                }
            }
        }
    }
}

// Sets the presence bit of every key of a seed table's n entries (the
// bitmap cleared before).
__global__ void seed_bitmap_kernel(const uint2 *ent, uint32_t n, uint32_t *bm, uint32_t key_bits)
{
    const uint32_t lanes = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += lanes) {
        const uint32_t bit = seed_bit(ent[i].x, key_bits);
        atomicOr(&bm[bit >> 5], 1u << (bit & 31u));
    }
}

// Clears counters on the stream (a kernel, so the launch sequence can be
// captured in a graph).
// ---------------------------------------------------------------------------
// Chunk expansion: the host uploads the hi and lo planes of a chunk's used
// words and a sorted list of the words whose N or piece-end bits are not
// all zero, (word, nm, em, 0); these kernels rebuild the dense nm and em
// planes, the padding words (hi = lo = 0, nm = em = all ones), and one flag
// byte per 32-word block: non-zero when the block holds an N bit or lies
// past the used words.
// ---------------------------------------------------------------------------

__global__ void expand_fill_kernel(uint32_t *hi, uint32_t *lo, uint32_t *nm, uint32_t *em,
                                   uint8_t *nflag, uint32_t used, uint32_t total,
                                   uint32_t blocks)
{
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < total; x += stride) {
        const uint32_t v = x < used ? 0u : 0xffffffffu;
        nm[x] = v;
        em[x] = v;
        if (x >= used) {
            hi[x] = 0u;
            lo[x] = 0u;
        }
    }
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < blocks; b += stride)
        nflag[b] = (32ull * b + 31u >= used) ? 1u : 0u;
}

__global__ void expand_scatter_kernel(uint32_t *nm, uint32_t *em, uint8_t *nflag,
                                      const uint4 *list, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 e = list[i];
    nm[e.x] = e.y;
    em[e.x] = e.z;
    if (e.y) nflag[e.x >> 5] = 1u;
}

__global__ void clear_u64_kernel(unsigned long long *p, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void clear_u32_kernel(unsigned int *p, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Static scratch for the allocation-free scan entry point: the pass counters
// (hit count, work count, skipped waves) and the filter work list of a pass,
// in a fixed device array instead of memory the context allocates. Every
// device holds its own copy. Host code reaches it only through the address
// hipGetSymbolAddress returns on that device (scratch_address): the array's
// name in host code is a host-side stand-in, not a device address.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];
}  // namespace

// Address of `scratch` on `device` (looked up once per device, with that
// device current); nullptr and the HIP error in *err when the lookup fails.
void *scratch_address(int device, hipError_t *err)
{
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipSetDevice(device);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) {
            *err = e;
            return nullptr;
        }
        g_scratch[device] = ptr;
    }
    return g_scratch[device];
}

// ---------------------------------------------------------------------------
// variant table
// ---------------------------------------------------------------------------

struct VariantDesc {
    void (*filter)(ScanArgs);
    void (*filter2)(ScanArgs);   // for query sets whose filter prefix spans two words
    void (*resolve)(ScanArgs);
    void (*dense)(ScanArgs);
    void (*dense_cold)(ScanArgs);
    uint32_t windows;   // W
    uint32_t qunroll;   // QU
    uint32_t wg;        // filter workgroup size
    uint32_t enc;       // filter arithmetic: 0 = VALU bit ops, 1 = fp4 matrix cores
                        // (four classes), 2 = fp4 matrix cores (three classes)
    uint32_t waves;     // matrix-core filter: waves launched over all batches
    uint32_t dmfma;     // 1: dense strands of at most 32 bases on the matrix cores
                        // (clean waves; three-class filters only)
};

#define IFA_V(W, QU, WG)                                                                 \
    {                                                                                    \
        scan_filter_kernel<W, QU, WG>, scan_filter_kernel<W, QU, WG>,                    \
            scan_resolve_kernel<W>, scan_dense_kernel<W>, scan_dense_cold_kernel<W>, W, QU,  \
            WG, 0, 0, 0                                                                  \
    }
// matrix-core filters: waves of 16 windows per lane, resolved by the W = 16 kernels
#define IFA_VM3(WG, WAVES)                                                               \
    {                                                                                    \
        scan_filter_mfma3_kernel<WG, 1>, scan_filter_mfma3_kernel<WG, 2>,                \
            scan_resolve_kernel<16>, scan_dense_kernel<16>, scan_dense_cold_kernel<16>, 16,  \
            4, WG, 2, WAVES, 0                                                           \
    }
// the same, with dense strands of at most 32 bases on the matrix cores
#define IFA_VM3D(WG, WAVES)                                                              \
    {                                                                                    \
        scan_filter_mfma3_kernel<WG, 1>, scan_filter_mfma3_kernel<WG, 2>,                \
            scan_resolve_kernel<16>, scan_dense_kernel<16>, scan_dense_cold_kernel<16>, 16,  \
            4, WG, 2, WAVES, 1                                                           \
    }
#define IFA_VM(WG, WAVES)                                                                \
    {                                                                                    \
        scan_filter_mfma_kernel<WG>, scan_filter_mfma_kernel<WG>, scan_resolve_kernel<16>, \
            scan_dense_kernel<16>, scan_dense_cold_kernel<16>, 16, 2, WG, 1, WAVES, 0    \
    }
static const VariantDesc kVariantTable[] = {
    IFA_V(32, 1, 256),   // 0
    IFA_V(32, 1, 64),    IFA_V(32, 1, 128),  IFA_V(32, 1, 512),
    IFA_V(32, 2, 256),   IFA_V(32, 2, 128),
    IFA_V(16, 1, 256),   IFA_V(16, 1, 128),  IFA_V(16, 1, 512),
    IFA_V(16, 2, 256),   IFA_V(16, 2, 512),
    IFA_V(32, 2, 512),   IFA_V(16, 2, 1024),
    IFA_VM(512, 32768),  IFA_VM(256, 32768),  IFA_VM(1024, 32768),
    IFA_VM(512, 16384),  IFA_VM(512, 65536),  IFA_VM(1024, 65536),
    IFA_VM3(512, 32768), IFA_VM3(256, 32768), IFA_VM3(1024, 32768),
    IFA_VM3(512, 65536), IFA_VM3(256, 16384),
    IFA_VM3D(256, 32768), IFA_VM3D(512, 32768), IFA_VM3D(512, 65536),
};
#undef IFA_V
#undef IFA_VM
#undef IFA_VM3
#undef IFA_VM3D

uint32_t variant_count() { return sizeof(kVariantTable) / sizeof(kVariantTable[0]); }

// Variant a context starts with: the three-class matrix-core filter with
// 256-thread workgroups (index of IFA_VM3(256, 32768) above).
uint32_t variant_default() { return 20; }

void variant_shape(uint32_t v, uint32_t *windows, uint32_t *qunroll, uint32_t *wg, uint32_t *enc)
{
    const VariantDesc &d = kVariantTable[v < variant_count() ? v : 0];
    *windows = d.windows;
    *qunroll = d.qunroll;
    *wg = d.wg;
    // encoding 3: the three-class filter with dense strands on the matrix cores
    *enc = d.enc + d.dmfma;
}

// Launch of a scan kernel, or (rec != nullptr) its record in a launch plan.
static hipError_t go(void (*f)(ScanArgs), dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                     const ScanArgs &a, std::vector<ScanLaunch> *rec)
{
    if (rec) {
        rec->push_back(ScanLaunch{reinterpret_cast<const void *>(f), grid, block, lds, a});
        return hipSuccess;
    }
    hipLaunchKernelGGL(f, grid, block, lds, s, a);
    return hipGetLastError();
}

static const VariantDesc &pick(const ScanArgs &a)
{
    return kVariantTable[a.variant < variant_count() ? a.variant : 0];
}

// Filter lanes of the word range (a multiple of 64, whole waves).
static uint64_t filter_lanes(const ScanArgs &a, const VariantDesc &v)
{
    const uint64_t lanes = (uint64_t)(a.w_end - a.w_begin) * (32u / v.windows);
    return (lanes + 63) & ~63ull;
}

// Sparse part, step 1: the filter kernel fills the work list (the caller
// clears *work_count and *skip_count first).
hipError_t launch_filter(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec)
{
    if (a.w_end <= a.w_begin || a.n_sparse == 0) return hipSuccess;
    const VariantDesc &v = pick(a);
    if (v.enc == 1 || v.enc == 2) {
        // about v.waves waves over all batches of 32 strands (grid y), at
        // most one per filter wave; each walks its share of the filter waves.
        // Three-class form: the leading batches that hold a two-word tile
        // run the two-word kernel, the rest the one-word kernel (more waves
        // per SIMD).
        const uint32_t waves = (a.w_end - a.w_begin + 31u) >> 5;
        const uint32_t wpg = v.wg / 64u;
        const uint32_t batches = (a.n_sparse + 31u) / 32u;
        const uint32_t want = (v.waves + wpg * batches - 1) / (wpg * batches);
        uint32_t gx = max(1u, min((waves + wpg - 1) / wpg, want));
        // a multiple of 8 lets the kernel give each XCD a contiguous run of
        // waves (xcd_local_x)
        if (gx >= 8u) gx &= ~7u;
        const uint32_t split =
            v.enc == 2 && a.mq3_words >= 2 ? min(a.mq3_two_batches, batches) : 0u;
        for (int part_nw = 2; part_nw >= 1; part_nw--) {
            const uint32_t lo = part_nw == 2 ? 0u : split, hi = part_nw == 2 ? split : batches;
            if (v.enc == 1 && part_nw == 2) continue;
            const bool two = part_nw == 2;
            const uint32_t lds =
                v.enc == 1 ? mq_lds_bytes(min(16u, (a.n_sparse + 1u) / 2u))
                           : mq3_lds_bytes(min(8u, (a.n_sparse + 3u) / 4u), v.wg, two ? 2 : 1);
            for (uint32_t b0 = lo; b0 < hi; b0 += 65535u) {
                ScanArgs part = a;
                part.batch0 = b0;
                const hipError_t e = go(two ? v.filter2 : v.filter,
                                        dim3(gx, min(65535u, hi - b0)), dim3(v.wg), lds, s, part, rec);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    }
    const uint64_t lanes = filter_lanes(a, v);
    return go(v.filter, dim3((uint32_t)((lanes + v.wg - 1) / v.wg)), dim3(v.wg), 0, s, a, rec);
}

// Sparse part, step 2: resolve the work list (a fixed grid, grid-stride).
hipError_t launch_resolve(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec)
{
    if (a.w_end <= a.w_begin || a.n_sparse == 0) return hipSuccess;
    return go(pick(a).resolve, dim3(1024), dim3(256), 0, s, a, rec);
}

// Dense part: query strands [n_sparse, n_qs) on every lane (plain lanes in
// the dense kernel, the others in the cold kernel).
hipError_t launch_dense(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec)
{
    if (a.w_end <= a.w_begin || a.n_qs <= a.n_sparse) return hipSuccess;
    const VariantDesc &v = pick(a);
    const uint64_t lanes = filter_lanes(a, v);
    const dim3 grid((uint32_t)((lanes + 255) / 256));
    // each side of the seam by L descending, in a launch of its own; with
    // the matrix kernel counting [dm_first = seam, n_qs) on clean waves, the
    // second launch takes only the waves it leaves out
    hipError_t e = hipSuccess;
    const uint32_t seam = a.dense_seam;
    if (seam > a.n_sparse) {
        ScanArgs part = a;
        part.dense_begin = a.n_sparse;
        part.dense_end = seam;
        e = go(v.dense, grid, dim3(256), 0, s, part, rec);
        if (e != hipSuccess) return e;
    }
    if (seam < a.n_qs) {
        ScanArgs part = a;
        part.dense_begin = seam;
        part.dense_end = a.n_qs;
        part.dense_unclean = a.dm_first < a.n_qs ? 1u : 0u;
        e = go(v.dense, grid, dim3(256), 0, s, part, rec);
        if (e != hipSuccess) return e;
    }
    e = go(v.dense_cold, grid, dim3(256), 0, s, a, rec);
    if (e != hipSuccess || a.dm_first >= a.n_qs) return e;
    // one-word dense strands on the matrix cores, clean waves only: one
    // batch of kDmTiles column tiles (4 kDmTiles strands) per grid row, about 2^15
    // waves in all
    const uint32_t tiles = (a.n_qs - a.dm_first + 3u) / 4u;
    const uint32_t batches = (tiles + kDmTiles - 1u) / kDmTiles;
    const uint32_t waves = (a.w_end - a.w_begin + 31u) >> 5;
    uint32_t gx = max(1u, min((waves + 3u) / 4u, (32768u / 4u + batches - 1u) / batches));
    if (gx >= 8u) gx &= ~7u;
    for (uint32_t b0 = 0; b0 < batches; b0 += 65535u) {
        ScanArgs part = a;
        part.dm_first = a.dm_first + 4u * kDmTiles * b0;
        part.dm_b = a.dm_b + 128u * kDmTiles * b0;
        part.dm_t = a.dm_t + 32u * kDmTiles * b0;
        e = go(scan_dense_mfma3_kernel<256>, dim3(gx, min(65535u, batches - b0)), dim3(256),
               dm3_lds_bytes(256), s, part, rec);
        if (e != hipSuccess) return e;
    }
    return e;
}

// Overhanging windows of the word range: one wave per (block of pieces,
// query strand) task, grid-stride.
hipError_t launch_edge(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec)
{
    if (a.w_end <= a.w_begin || a.n_pieces == 0 || a.n_qs == 0 || a.edge_pmin == 0)
        return hipSuccess;
    const uint64_t tasks = (uint64_t)((a.n_pieces + a.edge_pmin - 1) / a.edge_pmin) * a.n_qs;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((tasks + 3) / 4, 4096);
    return go(scan_edge_kernel, dim3(blocks), dim3(256), 0, s, a, rec);
}

// Indexed mode: seed starts of the word range, grid-stride.
hipError_t launch_seed(const ScanArgs &a, hipStream_t s, std::vector<ScanLaunch> *rec)
{
    if (a.w_end <= a.w_begin || a.seed_ncfg == 0) return hipSuccess;
    const uint32_t words = a.w_end - a.w_begin;
    const uint32_t blocks = std::min<uint32_t>((words + 255) / 256, 4096);
    return go(scan_seed_kernel, dim3(blocks), dim3(256), 0, s, a, rec);
}

// Rebuild a chunk's nm and em planes, padding and N-block flags from the
// sparse list (see expand_fill_kernel), on stream s after the planes' copy.
hipError_t launch_expand(uint32_t *planes, uint64_t stride, uint8_t *nflag, uint32_t used,
                         uint32_t total, const uint4 *list, uint32_t n_list, hipStream_t s)
{
    uint32_t *hi = planes, *lo = planes + stride, *nm = planes + 2 * stride, *em = planes + 3 * stride;
    const uint32_t blocks = nflag_blocks(total);
    const uint32_t grid = std::min<uint32_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(expand_fill_kernel, dim3(grid), dim3(256), 0, s, hi, lo, nm, em, nflag,
                       used, total, blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_list == 0) return e;
    hipLaunchKernelGGL(expand_scatter_kernel, dim3((n_list + 255) / 256), dim3(256), 0, s, nm, em,
                       nflag, list, n_list);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_clear_u32(unsigned int *p, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// Presence bitmap of a seed table: `words` 32-bit words (2^seed_bitmap_bits
// bits, at least one word) cleared, then one bit set per entry.
hipError_t launch_seed_bitmap(const uint2 *ent, uint32_t n, uint32_t *bm, uint32_t words,
                              uint32_t key_bits, hipStream_t s)
{
    hipError_t e = launch_clear_u32(bm, words, s);
    if (e != hipSuccess || n == 0) return e;
    const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(seed_bitmap_kernel, dim3(blocks), dim3(256), 0, s, ent, n, bm, key_bits);
    return hipGetLastError();
}

}  // namespace ifa
