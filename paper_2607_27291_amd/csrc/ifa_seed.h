// ifa_seed.h -- indexed mode, host side (see ifa_seed.cpp).
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "ifa_dev.h"

namespace ifa {

// Query count from which automatic mode selection picks indexed mode: the
// first count at which indexed mode's load + scan beat brute force's on the
// paper-scale 4 Gbp resident reference (queries of 30-36 bases, maxSubs 4).
constexpr uint32_t kAutoQueries = 100;

struct SeedParams {
    uint32_t n_k = 5;                                     // the paper's default lengths
    uint32_t k[kMaxSeedCfg] = {8, 9, 10, 12, 14, 0, 0, 0};
    uint32_t mask = 0;
    uint32_t step = 1;
    uint32_t ppm = 999000;
    uint64_t iters = 200000;
    uint64_t seed = 1;
    uint32_t auto_queries = kAutoQueries;
};

// Allocator whose value-less construct leaves the element uninitialised: the
// seed tables (hundreds of MB) are written whole after sizing, so zeroing
// them first would only cost time.
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = DefaultInitAlloc<U>;
    };
    DefaultInitAlloc() = default;
    template <class U>
    DefaultInitAlloc(const DefaultInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept
    {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a)
    {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
using TableBuf = std::vector<uint32_t, DefaultInitAlloc<uint32_t>>;

// MinHits results by (valid seeds, maxSubs, k) for the current parameters.
using MinHitsCache = std::map<std::tuple<uint32_t, uint32_t, uint32_t>, int64_t>;

struct SeedBuild {
    std::vector<SeedInfo> info;      // per query strand, in device order
    std::vector<uint32_t> qk;        // per query: seed length
    std::vector<uint32_t> qthr;      // per query and strand: threshold (0: not scanned)
    struct Cfg {
        uint32_t k = 0, bits = 0;
        TableBuf dir;                // 2^bits + 1 bucket starts
        TableBuf ent;                // (key, strand << 8 | offset) pairs
    };
    std::vector<Cfg> cfg;
};

uint32_t seed_keff(uint32_t k, uint32_t mask, uint32_t step);
int64_t seed_minhits(uint32_t V, uint32_t subs, uint32_t k, uint32_t mask, uint32_t step,
                     uint64_t iters, uint64_t seed, uint32_t ppm);

// qs/words: the context's query strands (device order) and their packed
// words; fwd_words/fwd_off: every query's forward strand packed the same way
// (words of query j start at fwd_off[j]).
void build_seeds(const SeedParams &P, uint32_t n_queries, const uint32_t *qlen,
                 const int32_t *max_subs, const std::vector<QSDesc> &qs,
                 const std::vector<uint32_t> &words, const std::vector<uint32_t> &fwd_words,
                 const std::vector<uint32_t> &fwd_off, unsigned threads, MinHitsCache &cache,
                 SeedBuild &out);

}  // namespace ifa
