// ifa_scan.hip -- gfx950 kernels of the brute-force gapless scan.
//
// Brute-force mode tests every start position of the reference against every
// query (Methods, "Algorithm Design"). The paper's CPU kernel compares one
// query base against 32 consecutive reference positions per vector step and
// keeps per-lane substitution and N ("clip") counters, stopping once every
// lane is past a threshold (Methods, "SIMD Optimization"). Here the reference
// is held as 2-bit bit planes and each GPU lane owns the 32 consecutive
// window starts of one plane word w:
//
//   * The lane loads plane words w and w+1 and forms, once, the 32 funnel
//     shifts (v_alignbit_b32) that give every one of its windows' first 32
//     bases as one word per plane. They are shared by every query and strand.
//   * Filter, per query strand: the mismatches of a window's first 32 bases
//     are popcount((qh ^ rh) | (ql ^ rl) | qn), two v_bitop3_b32 and one
//     v_bcnt_u32_b32, folded over the lane's 32 windows with v_min3_u32.
//     Query bits at or past L are zero and are not masked, so those positions
//     can add up to 32 - min(L, 32) to the count; a window can be a hit only
//     if this count is <= k + 32 - min(L, 32). When no window of the lane
//     passes (almost always), the lane is done with this query: the paper's
//     early exit, taken per 32 bases.
//   * Reference N positions must not count in the filter; waves whose bases
//     hold an N (rare) run the filter with the N positions masked out.
//   * Windows that pass go to the exact test, which walks every query word
//     and applies the N rule, piece boundaries and chunk ownership.
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

// Three-input bitwise op (v_bitop3_b32): bit i of the result is bit
// (a_i << 2 | b_i << 1 | c_i) of the truth table `tt`.
#define IFA_XOR_OR 0xBEu   // (a ^ b) | c
#define IFA_OR_XOR 0xF6u   // a | (b ^ c)

// A query strand descriptor, unpacked from one 16-byte scalar load.
struct QS {
    uint32_t qid, len, strand, nw, k, maxn, woff;
};

__device__ __forceinline__ QS load_qs(const ScanArgs &a, uint32_t q)
{
    const IFA_CONST uint32_t *r = as_const(reinterpret_cast<const uint32_t *>(a.qs)) + 4u * q;
    const uint32_t r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
    QS d;
    d.qid = r0;
    d.len = r1 & 0xffffu;
    d.strand = (r1 >> 16) & 0xffu;
    d.nw = r1 >> 24;
    d.k = r2 & 0xffffu;
    d.maxn = r2 >> 16;
    d.woff = r3;
    return d;
}

__device__ __forceinline__ uint64_t splitmix_fin(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Map a chunk position to (contig ordinal, contig coordinate) and record it.
__device__ void emit_hit(const ScanArgs &a, const QS &d, uint64_t p, uint32_t m,
                         uint32_t nref)
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
            rec.w = (uint32_t)d.strand | (nref << 8) | (m << 16);
            a.hits[slot] = rec;
        }
    } else {
        const uint64_t key = ((uint64_t)contig << 32) | pos;
        const uint64_t aux = (uint64_t)d.strand | ((uint64_t)m << 1) | ((uint64_t)nref << 10);
        atomicAdd(&a.q_count[d.qid], 1ull);
        atomicAdd(&a.q_digest[d.qid], (unsigned long long)splitmix_fin(key ^ (aux << 45)));
    }
}

// Exact test of the 32 windows starting in word w against one query strand.
__device__ __forceinline__ void exact_lane(const ScanArgs &a, const QS &d, uint32_t w)
{
    const uint32_t L = d.len;
    const IFA_CONST uint32_t *qw = as_const(a.qwords) + d.woff;
    for (uint32_t b = 0; b < 32; b++) {
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

// Filter every query strand against the lane's 32 windows; run the exact test
// where a window may be a hit. kMaskN: leave reference N positions out of the
// filter count (needed only when the wave's bases contain an N).
template <bool kMaskN>
__device__ __forceinline__ void scan_lane(const ScanArgs &a, uint32_t w, bool active,
                                          uint32_t h0, uint32_t h1, uint32_t l0, uint32_t l1,
                                          uint32_t n0, uint32_t n1)
{
    uint32_t sh[32], sl[32];
#pragma unroll
    for (int b = 0; b < 32; b++) {
        sh[b] = funnel(h1, h0, (uint32_t)b);
        sl[b] = funnel(l1, l0, (uint32_t)b);
    }
    const IFA_CONST uint32_t *qwords = as_const(a.qwords);
    for (uint32_t q = 0; q < a.n_qs; q++) {
        const QS d = load_qs(a, q);
        const uint32_t qh = qwords[d.woff], ql = qwords[d.woff + 1], qn = qwords[d.woff + 2];
        const uint32_t thr = d.k + 32u - min(d.len, 32u);
        bool cand = true;
        if (thr < 32u) {
            uint32_t mn = 0xffffffffu;
#pragma unroll
            for (int b = 0; b < 32; b++) {
                uint32_t diff = __builtin_amdgcn_bitop3_b32(sh[b], qh, qn, IFA_XOR_OR);
                diff = __builtin_amdgcn_bitop3_b32(diff, sl[b], ql, IFA_OR_XOR);
                if (kMaskN) diff &= ~funnel(n1, n0, (uint32_t)b);
                mn = min(mn, (uint32_t)__popc(diff));
            }
            cand = mn <= thr;
        }
        if (active && cand) exact_lane(a, d, w);
    }
}

__global__ __launch_bounds__(256) void scan_words_kernel(ScanArgs a)
{
    const uint32_t w = a.w_begin + blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = w < a.w_end;
    const uint32_t wl = active ? w : a.w_begin;

    const uint32_t h0 = a.hi[wl], h1 = a.hi[wl + 1];
    const uint32_t l0 = a.lo[wl], l1 = a.lo[wl + 1];
    const uint32_t n0 = a.nm[wl], n1 = a.nm[wl + 1];

    // Does any base of the lane's 32 windows (up to the first 32 bases of
    // each) hold an N? Words w and w+1 cover them.
    const bool lane_n = active && ((n0 | n1) != 0u);
    if (__any(lane_n))
        scan_lane<true>(a, w, active, h0, h1, l0, l1, n0, n1);
    else
        scan_lane<false>(a, w, active, h0, h1, l0, l1, n0, n1);
}

// Clears counters on the stream (a kernel, so the launch sequence can be
// captured in a graph).
__global__ void clear_u64_kernel(unsigned long long *p, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_scan(const ScanArgs &a, hipStream_t s)
{
    if (a.w_end <= a.w_begin || a.n_qs == 0) return hipSuccess;
    const uint32_t n = a.w_end - a.w_begin;
    const uint32_t block = 256;
    const uint32_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(scan_words_kernel, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(clear_u64_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace ifa
