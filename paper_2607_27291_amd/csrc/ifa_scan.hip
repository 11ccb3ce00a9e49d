// ifa_scan.hip -- gfx950 kernels of the brute-force gapless scan.
//
// Brute-force mode tests every start position of the reference against every
// query (Methods, "Algorithm Design"). The paper's CPU kernel compares one
// query base against 32 consecutive reference positions per vector step and
// keeps per-lane substitution and N ("clip") counters, stopping once every
// lane is past a threshold (Methods, "SIMD Optimization"). Here the reference
// is held as 2-bit bit planes and each GPU lane owns W consecutive window
// starts (W = 32: one plane word; W = 16: half a word):
//
//   * The lane loads plane words w and w+1 and forms, once, the W funnel
//     shifts (v_alignbit_b32) that give each of its windows' first 32 bases
//     as one word per plane. They are shared by every query and strand.
//   * Filter, per query strand: the mismatches of a window's first 32 bases
//     are popcount((qh ^ rh) | (ql ^ rl) | qn), two v_bitop3_b32 and one
//     v_bcnt_u32_b32, folded over the lane's windows with v_min3_u32.
//     Query bits at or past L are zero and are not masked, so those positions
//     can add up to 32 - min(L, 32) to the count; a window can be a hit only
//     if this count is <= thr = k + 32 - min(L, 32). When no window of the
//     lane passes (almost always), the lane is done with this query strand:
//     the paper's early exit, taken per 32 bases.
//   * Reference N positions must not count in the filter; waves whose bases
//     hold an N (rare) run the filter with the N positions masked out.
//   * Windows that pass go to the exact test, which walks every query word
//     and applies the N rule, piece boundaries and chunk ownership.
//
// Variants (template parameters, chosen by the autotuner): windows per lane
// W, query strands per loop iteration QU, and workgroup size.
#include <hip/hip_runtime.h>

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

// Map a chunk position to (contig ordinal, contig coordinate) and record it.
__device__ void emit_hit(const ScanArgs &a, const QS &d, uint64_t p, uint32_t m, uint32_t nref)
{
    uint32_t lo = 0, hi = a.n_pieces;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (a.pieces[mid].start <= p) lo = mid; else hi = mid;
    }
    const Piece pc = a.pieces[lo];
    const uint32_t contig = pc.contig;
    const uint32_t pos = (uint32_t)(pc.contig_off + (p - pc.start));
    if (a.sink == kSinkRecords) {
        unsigned long long slot = atomicAdd(a.hit_count, 1ull);
        if (slot < a.hit_cap) {
            uint4 rec;
            rec.x = d.qid;
            rec.y = contig;
            rec.z = pos;
            rec.w = d.strand | (nref << 8) | (m << 16);
            a.hits[slot] = rec;
        }
    } else {
        const uint64_t key = ((uint64_t)contig << 32) | pos;
        const uint64_t aux = (uint64_t)d.strand | ((uint64_t)m << 1) | ((uint64_t)nref << 10);
        atomicAdd(&a.q_count[d.qid], 1ull);
        atomicAdd(&a.q_digest[d.qid], (unsigned long long)splitmix_fin(key ^ (aux << 45)));
    }
}

// Exact test of windows 32w + off .. 32w + off + W - 1 against one query strand.
template <int W>
__device__ __forceinline__ void exact_lane(const ScanArgs &a, const QS &d, uint32_t w,
                                           uint32_t off)
{
    const uint32_t L = d.len;
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    for (uint32_t b = off; b < off + (uint32_t)W; b++) {
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
        emit_hit(a, d, p, m, nref);
    }
}

// Minimum over the lane's W windows of the filter count for one query strand.
template <int W, bool kMaskN>
__device__ __forceinline__ uint32_t filter_min(const uint32_t (&sh)[W], const uint32_t (&sl)[W],
                                               const QS &d, uint32_t n0, uint32_t n1, uint32_t off)
{
    uint32_t mn = 0xffffffffu;
#pragma unroll
    for (int b = 0; b < W; b++) {
        uint32_t diff = __builtin_amdgcn_bitop3_b32(sh[b], d.qh, d.qn, IFA_XOR_OR);
        diff = __builtin_amdgcn_bitop3_b32(diff, sl[b], d.ql, IFA_OR_XOR);
        if (kMaskN) diff &= ~funnel(n1, n0, off + (uint32_t)b);
        mn = min(mn, (uint32_t)__popc(diff));
    }
    return mn;
}

// Filter every query strand against the lane's W windows; run the exact test
// where a window may be a hit.
template <int W, int QU, bool kMaskN>
__device__ __forceinline__ void scan_lane(const ScanArgs &a, uint32_t w, uint32_t off,
                                          bool active, uint32_t h0, uint32_t h1, uint32_t l0,
                                          uint32_t l1, uint32_t n0, uint32_t n1)
{
    uint32_t sh[W], sl[W];
#pragma unroll
    for (int b = 0; b < W; b++) {
        sh[b] = funnel(h1, h0, off + (uint32_t)b);
        sl[b] = funnel(l1, l0, off + (uint32_t)b);
    }
    const uint32_t n = a.n_qs;
    uint32_t q = 0;
    if (QU == 2) {
        for (; q + 1 < n; q += 2) {
            const QS d0 = load_qs(a, q);
            const QS d1 = load_qs(a, q + 1);
            const bool c0 =
                d0.thr >= 32u || filter_min<W, kMaskN>(sh, sl, d0, n0, n1, off) <= d0.thr;
            const bool c1 =
                d1.thr >= 32u || filter_min<W, kMaskN>(sh, sl, d1, n0, n1, off) <= d1.thr;
            if (active && c0) exact_lane<W>(a, d0, w, off);
            if (active && c1) exact_lane<W>(a, d1, w, off);
        }
    }
    for (; q < n; q++) {
        const QS d = load_qs(a, q);
        const bool c = d.thr >= 32u || filter_min<W, kMaskN>(sh, sl, d, n0, n1, off) <= d.thr;
        if (active && c) exact_lane<W>(a, d, w, off);
    }
}

template <int W, int QU, int WG>
__global__ __launch_bounds__(WG) void scan_kernel(ScanArgs a)
{
    constexpr uint32_t kLanesPerWord = 32 / W;
    const uint32_t lane = blockIdx.x * WG + threadIdx.x;
    const uint32_t w = a.w_begin + lane / kLanesPerWord;
    const uint32_t off = (lane % kLanesPerWord) * (uint32_t)W;
    const bool active = w < a.w_end;
    const uint32_t wl = active ? w : a.w_begin;

    const uint32_t h0 = a.hi[wl], h1 = a.hi[wl + 1];
    const uint32_t l0 = a.lo[wl], l1 = a.lo[wl + 1];
    const uint32_t n0 = a.nm[wl], n1 = a.nm[wl + 1];

    // Does any base the filter reads for this lane hold an N? Words w and
    // w+1 cover the first 32 bases of all of the lane's windows.
    const bool lane_n = active && ((n0 | n1) != 0u);
    if (__any(lane_n))
        scan_lane<W, QU, true>(a, w, off, active, h0, h1, l0, l1, n0, n1);
    else
        scan_lane<W, QU, false>(a, w, off, active, h0, h1, l0, l1, n0, n1);
}

// Clears counters on the stream (a kernel, so the launch sequence can be
// captured in a graph).
__global__ void clear_u64_kernel(unsigned long long *p, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// variant table
// ---------------------------------------------------------------------------

struct VariantDesc {
    void (*fn)(ScanArgs);
    uint32_t windows;   // W
    uint32_t qunroll;   // QU
    uint32_t wg;        // workgroup size
};

#define IFA_V(W, QU, WG) { scan_kernel<W, QU, WG>, W, QU, WG }
static const VariantDesc kVariantTable[] = {
    IFA_V(32, 1, 256),   // 0: default
    IFA_V(32, 1, 64),    IFA_V(32, 1, 128),  IFA_V(32, 1, 512),
    IFA_V(32, 2, 256),   IFA_V(32, 2, 128),
    IFA_V(16, 1, 256),   IFA_V(16, 1, 128),  IFA_V(16, 1, 512),
    IFA_V(16, 2, 256),   IFA_V(16, 2, 512),
};
#undef IFA_V

uint32_t variant_count() { return sizeof(kVariantTable) / sizeof(kVariantTable[0]); }

void variant_shape(uint32_t v, uint32_t *windows, uint32_t *qunroll, uint32_t *wg)
{
    const VariantDesc &d = kVariantTable[v < variant_count() ? v : 0];
    *windows = d.windows;
    *qunroll = d.qunroll;
    *wg = d.wg;
}

hipError_t launch_scan(const ScanArgs &a, hipStream_t s)
{
    if (a.w_end <= a.w_begin || a.n_qs == 0) return hipSuccess;
    const VariantDesc &v = kVariantTable[a.variant < variant_count() ? a.variant : 0];
    const uint64_t lanes = (uint64_t)(a.w_end - a.w_begin) * (32u / v.windows);
    const uint64_t grid = (lanes + v.wg - 1) / v.wg;
    hipLaunchKernelGGL(v.fn, dim3((uint32_t)grid), dim3(v.wg), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace ifa
