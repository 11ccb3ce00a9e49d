// ifa_seed.cpp -- indexed mode, host side: seed length per query, MinHits per
// query strand, and the device seed tables (Methods, "Algorithm Design").
//
// Seeds of a query strand are its k-mers at offsets 0, step, 2 step, ... with
// no N at an unmasked position (a centre of `mask` bases is ignored). MinHits
// is the number of error-free seeds a valid alignment keeps with probability
// prob_ppm / 10^6, by Monte Carlo over substitution placements, or the
// deterministic bound V - kEffective x maxSubs at probability 1. The seed
// length is the longest candidate whose MinHits is at least 1.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <thread>
#include <tuple>
#include <vector>

#include "ifa_seed.h"

namespace ifa {
namespace {

// SplitMix64 (Steele, Lea & Flood 2014): draw n of the stream `seed` is the
// output finaliser applied to seed + (n + 1) * the golden gamma.
inline uint64_t splitmix_draw(uint64_t seed, uint64_t n)
{
    uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Uniform integer in [0, m) from a 64-bit draw: high half of draw * m
// (Lemire's multiply-shift).
inline uint32_t below(uint64_t draw, uint32_t m)
{
    return (uint32_t)(((unsigned __int128)draw * m) >> 64);
}

inline bool unmasked(uint32_t t, uint32_t k, uint32_t mask)
{
    const uint32_t lo = (k - mask) / 2;
    return t < lo || t >= lo + mask;
}

}  // namespace

uint32_t seed_keff(uint32_t k, uint32_t mask, uint32_t step)
{
    // seeds one base can touch at an unmasked offset; the count repeats
    // with period `step` once the base is k - 1 or more bases in
    uint32_t best = 0;
    for (uint32_t x = 0; x < k + step * k; x++) {
        uint32_t c = 0;
        for (uint32_t v = 0; v * step <= x; v++)
            if (x - v * step < k && unmasked(x - v * step, k, mask)) c++;
        best = std::max(best, c);
    }
    return best;
}

int64_t seed_minhits(uint32_t V, uint32_t subs, uint32_t k, uint32_t mask, uint32_t step,
                     uint64_t iters, uint64_t seed, uint32_t ppm)
{
    if (V == 0) return 0;
    const uint32_t span = (V - 1) * step + k;
    const uint32_t s = std::min(subs, span);
    if (ppm >= 1000000u) return (int64_t)V - (int64_t)seed_keff(k, mask, step) * s;
    if (s == 0) return V;   // every trial keeps all V seeds
    std::vector<uint32_t> perm(span), hit(V, 0);
    for (uint32_t i = 0; i < span; i++) perm[i] = i;
    std::vector<uint64_t> hist(V + 1, 0);
    uint64_t n = 0;
    for (uint64_t trial = 1; trial <= iters; trial++) {
        // partial Fisher-Yates: slot c takes a uniform slot of [c, span)
        for (uint32_t c = 0; c < s; c++) {
            const uint32_t j = c + below(splitmix_draw(seed, n++), span - c);
            std::swap(perm[c], perm[j]);
        }
        // seeds v with an unmasked offset on a substituted base die; hit[v]
        // holds the last trial that killed v
        uint32_t dead = 0;
        for (uint32_t c = 0; c < s; c++) {
            const uint32_t x = perm[c];
            const uint32_t vlo = x >= k ? (x - k) / step + 1 : 0;   // v step > x - k
            const uint32_t vhi = std::min(V - 1, x / step);
            for (uint32_t v = vlo; v <= vhi && vlo <= vhi; v++) {
                if (!unmasked(x - v * step, k, mask) || hit[v] == (uint32_t)trial) continue;
                hit[v] = (uint32_t)trial;
                dead++;
            }
        }
        hist[V - dead]++;
    }
    uint64_t acc = 0;
    for (int64_t t = V; t >= 0; t--) {
        acc += hist[(size_t)t];
        if ((unsigned __int128)acc * 1000000u >= (unsigned __int128)ppm * iters) return t;
    }
    return 0;
}

namespace {

// bits [i, i + n) (n <= 32) of plane `pl` of a strand packed as 32-bit
// words (hi, lo, qn) x nw
inline uint32_t bits_at(const uint32_t *w3, uint32_t nw, uint32_t pl, uint32_t i, uint32_t n)
{
    const uint32_t a = i >> 5, sh = i & 31u;
    uint64_t v = w3[3 * a + pl];
    if (a + 1 < nw) v |= (uint64_t)w3[3 * (a + 1) + pl] << 32;
    v >>= sh;
    return n >= 32 ? (uint32_t)v : (uint32_t)v & ((1u << n) - 1u);
}

inline uint32_t squeeze(uint32_t x, uint32_t k, uint32_t mask)
{
    const uint32_t lo = (k - mask) / 2;
    return (x & ((1u << lo) - 1u)) | ((x >> (lo + mask)) << lo);
}

// Seed of a strand (planes hi, lo, qn as 32-bit words, stride 3) at offset i:
// false if it holds an N at an unmasked position, else its key.
bool strand_seed(const uint32_t *w3, uint32_t nw, uint32_t i, uint32_t k, uint32_t mask,
                 uint32_t *key)
{
    if (squeeze(bits_at(w3, nw, 2, i, k), k, mask) != 0u) return false;
    const uint32_t u = k - mask;
    *key = (squeeze(bits_at(w3, nw, 0, i, k), k, mask) << u) |
           squeeze(bits_at(w3, nw, 1, i, k), k, mask);
    return true;
}

uint32_t count_seeds(const uint32_t *w3, uint32_t nw, uint32_t L, uint32_t k, uint32_t mask,
                     uint32_t step)
{
    uint32_t n = 0, key;
    for (uint32_t i = 0; i + k <= L; i += step) n += strand_seed(w3, nw, i, k, mask, &key);
    return n;
}

using Tuple = std::tuple<uint32_t, uint32_t, uint32_t>;   // (V, subs, k)

// f(i) for i in [0, n) on up to `threads` threads, in contiguous blocks
template <class F>
void parallel_for(size_t n, unsigned threads, F &&f)
{
    const unsigned nt = (unsigned)std::max<size_t>(1, std::min<size_t>(threads, n / 256 + 1));
    std::vector<std::thread> pool;
    auto run = [&](unsigned t) {
        const size_t a = n * t / nt, b = n * (t + 1) / nt;
        for (size_t i = a; i < b; i++) f(i);
    };
    for (unsigned t = 1; t < nt; t++) pool.emplace_back(run, t);
    run(0);
    for (auto &th : pool) th.join();
}

// f(b) for every block b in [0, nb), blocks handed out one at a time to up to
// `threads` threads
template <class F>
void parallel_blocks(size_t nb, unsigned threads, F &&f)
{
    const unsigned nt = (unsigned)std::max<size_t>(1, std::min<size_t>(threads, nb));
    std::atomic<size_t> next{0};
    auto run = [&]() {
        for (size_t b; (b = next.fetch_add(1)) < nb;) f(b);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; t++) pool.emplace_back(run);
    run();
    for (auto &th : pool) th.join();
}

// Stable counting sort of (keys[e], tags[e]) into buckets (key * golden) >>
// (32 - bits): dir[b] = first entry of bucket b, dir[2^bits] = n; ent holds
// (key, tag) pairs, a bucket's entries in input order. Two passes, both
// parallel: a partition by the top bits of the bucket (per-slice counts, so
// each slice scatters in input order), then each partition sorted on its own.
void bucket_sort(const TableBuf &keys, const TableBuf &tags, uint32_t bits, unsigned threads,
                 TableBuf &dir, TableBuf &ent)
{
    const size_t n = keys.size();
    const uint32_t sh = 32 - bits;
    const uint32_t pbits = std::min<uint32_t>(bits, 8), nparts = 1u << pbits;
    const uint32_t lbits = bits - pbits;              // bucket bits inside a partition
    auto bucket = [&](uint32_t key) { return (key * 0x9E3779B1u) >> sh; };
    const size_t nslices = std::max<size_t>(1, std::min<size_t>(4 * threads, n / 4096 + 1));
    // per slice and partition: entry count, then scatter offset
    std::vector<size_t> off(nslices * nparts, 0);
    parallel_blocks(nslices, threads, [&](size_t t) {
        size_t *o = off.data() + t * nparts;
        for (size_t e = n * t / nslices; e < n * (t + 1) / nslices; e++) o[bucket(keys[e]) >> lbits]++;
    });
    std::vector<size_t> pstart(nparts + 1, 0);
    size_t acc = 0;
    for (uint32_t p = 0; p < nparts; p++) {
        pstart[p] = acc;
        for (size_t t = 0; t < nslices; t++) {
            const size_t c = off[t * nparts + p];
            off[t * nparts + p] = acc;
            acc += c;
        }
    }
    pstart[nparts] = acc;
    TableBuf k2(n), t2(n);
    parallel_blocks(nslices, threads, [&](size_t t) {
        size_t *o = off.data() + t * nparts;
        for (size_t e = n * t / nslices; e < n * (t + 1) / nslices; e++) {
            const size_t at = o[bucket(keys[e]) >> lbits]++;
            k2[at] = keys[e];
            t2[at] = tags[e];
        }
    });
    dir.resize(((size_t)1 << bits) + 1);   // every bucket start is written below
    ent.resize(2 * n);
    parallel_blocks(nparts, threads, [&](size_t p) {
        const size_t lo = pstart[p], hi = pstart[p + 1];
        const uint32_t b0 = (uint32_t)p << lbits, nb = 1u << lbits;
        std::vector<uint32_t> cnt(nb + 1, 0);
        for (size_t e = lo; e < hi; e++) cnt[bucket(k2[e]) - b0 + 1]++;
        for (uint32_t b = 0; b < nb; b++) cnt[b + 1] += cnt[b];
        for (uint32_t b = 0; b < nb; b++) dir[b0 + b] = (uint32_t)(lo + cnt[b]);
        for (size_t e = lo; e < hi; e++) {
            const size_t at = lo + cnt[bucket(k2[e]) - b0]++;
            ent[2 * at] = k2[e];
            ent[2 * at + 1] = t2[e];
        }
    });
    dir[(size_t)1 << bits] = (uint32_t)n;
}

}  // namespace

void build_seeds(const SeedParams &P, uint32_t n_queries, const uint32_t *qlen,
                 const int32_t *max_subs, const std::vector<QSDesc> &qs,
                 const std::vector<uint32_t> &words, const std::vector<uint32_t> &fwd_words,
                 const std::vector<uint32_t> &fwd_off, unsigned threads, MinHitsCache &cache,
                 SeedBuild &out)
{
    // MinHits for a batch of (V, subs, k), through the cache, on `threads`
    auto resolve = [&](const std::vector<Tuple> &want) {
        std::vector<Tuple> todo;
        for (const Tuple &t : want)
            if (std::get<0>(t) > 0 && !cache.count(t)) todo.push_back(t);
        std::sort(todo.begin(), todo.end());
        todo.erase(std::unique(todo.begin(), todo.end()), todo.end());
        std::vector<int64_t> res(todo.size());
        std::atomic<size_t> next{0};
        auto work = [&]() {
            for (size_t i; (i = next.fetch_add(1)) < todo.size();) {
                const Tuple &t = todo[i];
                res[i] = seed_minhits(std::get<0>(t), std::get<1>(t), std::get<2>(t), P.mask,
                                      P.step, P.iters, P.seed, P.ppm);
            }
        };
        const unsigned nt = std::max(1u, std::min<unsigned>(threads, (unsigned)todo.size()));
        std::vector<std::thread> pool;
        for (unsigned t = 1; t < nt; t++) pool.emplace_back(work);
        work();
        for (auto &th : pool) th.join();
        for (size_t i = 0; i < todo.size(); i++) cache[todo[i]] = res[i];
    };
    auto minhits = [&](uint32_t V, uint32_t s, uint32_t k) -> int64_t {
        return V == 0 ? 0 : cache.at(Tuple(V, s, k));
    };

    // candidate lengths, longest first
    std::vector<uint32_t> ks(P.k, P.k + P.n_k);
    std::sort(ks.rbegin(), ks.rend());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());

    // seed length per query: the longest candidate with MinHits >= 1 on the
    // forward strand, else the shortest; k = L below every candidate. The
    // tries run as rounds over all undecided queries so each round's MinHits
    // are computed in parallel.
    out.qk.assign(n_queries, 0);
    std::vector<std::vector<uint32_t>> cand(n_queries);
    std::vector<size_t> at(n_queries, 0);
    std::vector<uint32_t> subs(n_queries);
    for (uint32_t j = 0; j < n_queries; j++) {
        subs[j] = (uint32_t)std::min<int64_t>(max_subs[j], qlen[j]);
        for (uint32_t k : ks)
            if (k <= qlen[j] && k > P.mask) cand[j].push_back(k);
        if (cand[j].empty()) cand[j].push_back(qlen[j]);
    }
    auto fwd_valid = [&](uint32_t j, uint32_t k) {
        const uint32_t nw = (qlen[j] + 31) / 32;
        return count_seeds(fwd_words.data() + fwd_off[j], nw, qlen[j], k, P.mask, P.step);
    };
    std::vector<uint32_t> vcur(n_queries);   // forward seeds at the current try
    for (;;) {
        parallel_for(n_queries, threads, [&](size_t j) {
            if (!out.qk[j]) vcur[j] = fwd_valid((uint32_t)j, cand[j][at[j]]);
        });
        std::vector<Tuple> want;
        for (uint32_t j = 0; j < n_queries; j++)
            if (!out.qk[j]) want.emplace_back(vcur[j], subs[j], cand[j][at[j]]);
        if (want.empty()) break;
        resolve(want);
        for (uint32_t j = 0; j < n_queries; j++) {
            if (out.qk[j]) continue;
            const uint32_t k = cand[j][at[j]];
            if (minhits(vcur[j], subs[j], k) >= 1 || at[j] + 1 == cand[j].size())
                out.qk[j] = k;
            else
                at[j]++;
        }
    }

    // per strand: seeds, threshold max(1, MinHits of its own seed count)
    out.info.assign(qs.size(), SeedInfo{});
    out.qthr.assign(2 * (size_t)n_queries, 0);
    std::vector<uint32_t> nvalid(qs.size());
    parallel_for(qs.size(), threads, [&](size_t q) {
        const QSDesc &d = qs[q];
        SeedInfo &si = out.info[q];
        si.k = out.qk[d.qid];
        uint32_t key, n = 0;
        for (uint32_t i = 0; i + si.k <= d.len; i += P.step)
            if (strand_seed(words.data() + d.woff, d.nw, i, si.k, P.mask, &key)) {
                si.valid[i >> 5] |= 1u << (i & 31);
                n++;
            }
        nvalid[q] = n;
    });
    std::vector<Tuple> want;
    for (size_t q = 0; q < qs.size(); q++) want.emplace_back(nvalid[q], subs[qs[q].qid], out.info[q].k);
    resolve(want);
    for (size_t q = 0; q < qs.size(); q++) {
        const QSDesc &d = qs[q];
        out.info[q].thr = (uint32_t)std::max<int64_t>(1, minhits(nvalid[q], subs[d.qid], out.info[q].k));
        out.qthr[2 * (size_t)d.qid + d.strand] = out.info[q].thr;
    }

    // one table per distinct seed length
    std::map<uint32_t, size_t> slot;
    out.cfg.clear();
    for (size_t q = 0; q < qs.size(); q++) {
        if (!slot.count(out.info[q].k)) {
            slot[out.info[q].k] = out.cfg.size();
            out.cfg.emplace_back();
            out.cfg.back().k = out.info[q].k;
        }
    }
    for (auto &c : out.cfg) {
        // entries grouped by bucket (a counting sort), strand then offset
        // order inside a bucket
        size_t n_ent = 0;
        for (size_t q = 0; q < qs.size(); q++)
            if (out.info[q].k == c.k)
                for (uint32_t t = 0; t < kMaxQWords; t++)
                    n_ent += (size_t)__builtin_popcount(out.info[q].valid[t]);
        uint32_t bits = 4;
        while (bits < 24 && (1ull << bits) < 2 * n_ent) bits++;
        c.bits = bits;
        // keys of every seed of this length, strands in order (each strand's
        // slice located by a prefix sum of its seed count), in parallel
        std::vector<size_t> first(qs.size() + 1, 0);
        for (size_t q = 0; q < qs.size(); q++)
            first[q + 1] = first[q] + (out.info[q].k == c.k ? nvalid[q] : 0);
        TableBuf keys(n_ent), tags(n_ent);
        parallel_for(qs.size(), threads, [&](size_t q) {
            if (out.info[q].k != c.k) return;
            const QSDesc &d = qs[q];
            size_t at_ = first[q];
            uint32_t key;
            for (uint32_t i = 0; i + c.k <= d.len; i += P.step)
                if (strand_seed(words.data() + d.woff, d.nw, i, c.k, P.mask, &key)) {
                    keys[at_] = key;
                    tags[at_++] = ((uint32_t)q << 8) | i;
                }
        });
        bucket_sort(keys, tags, bits, threads, c.dir, c.ent);
    }
}

}  // namespace ifa
