// ifa_sam.cpp -- SAM text for hit records (host code, no device work).
//
// The aligner streams the reference, so its SAM output is headerless and a
// separate header is concatenated in front of it (Methods, "Output Format").
// A query's primary alignment is its first valid alignment in reference
// order; the others are secondary (Results, "Accuracy Validation"). Field
// choices where the paper is silent (SAM v1.6 meanings):
//   FLAG 16 for the reverse-complement strand, | 256 when secondary;
//   POS the 1-based first aligned base; MAPQ 255; CIGAR [aS]mM[bS] with a, b
//   the bases off the contig's left / right end (overhanging windows);
//   RNEXT *, PNEXT 0, TLEN 0; SEQ the strand sequence as compared (upper
//   case, N for non-ACGT); QUAL *; NM:i mismatches over the aligned bases,
//   XN:i reference Ns over the aligned bases.
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ifa.h"

struct ifa_sam {
    uint32_t policy = IFA_N_SEPARATE;
    std::vector<std::string> qname;
    std::vector<std::string> fwd, rev;     // strand sequences
    std::vector<uint8_t> seen;             // query already had its primary line
    std::vector<std::string> cname;
    std::vector<uint64_t> clen;
    bool have_last = false;
    ifa_hit last{};
    std::string err;
};

namespace {

char norm_base(uint8_t b)
{
    switch (b) {
    case 'A': case 'a': return 'A';
    case 'C': case 'c': return 'C';
    case 'G': case 'g': return 'G';
    case 'T': case 't': return 'T';
    default: return 'N';
    }
}

char comp_base(char c)
{
    switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    default: return 'N';
    }
}

bool clean_name(const char *s)
{
    if (!s || !*s) return false;
    for (; *s; s++)
        if (*s == '\t' || *s == '\n' || *s == '\r') return false;
    return true;
}

void put_u64(std::string &o, uint64_t v)
{
    char t[24];
    int n = 0;
    do {
        t[n++] = (char)('0' + v % 10);
        v /= 10;
    } while (v);
    while (n) o.push_back(t[--n]);
}

void put_i64(std::string &o, int64_t v)
{
    if (v < 0) {
        o.push_back('-');
        put_u64(o, (uint64_t)(-v));
    } else {
        put_u64(o, (uint64_t)v);
    }
}

// (contig, pos, strand, query) order
bool before(const ifa_hit &a, const ifa_hit &b)
{
    if (a.contig != b.contig) return a.contig < b.contig;
    if (a.pos != b.pos) return a.pos < b.pos;
    if (a.strand != b.strand) return a.strand < b.strand;
    return a.query < b.query;
}

}  // namespace

static ifa_status format_hits(ifa_sam *w, const ifa_hit *hits, uint64_t n, char *buf,
                              uint64_t cap, uint64_t *n_consumed, uint64_t *n_bytes);

extern "C" {

ifa_status ifa_sam_create(uint32_t n_queries, const uint8_t *const *seq, const uint32_t *len,
                          const char *const *names, uint32_t n_policy, ifa_sam **out)
{
    if (!out) return IFA_E_INVALID;
    *out = nullptr;
    if (n_policy > IFA_N_AS_MISMATCH) return IFA_E_INVALID;
    if (n_queries > 0 && (!seq || !len || !names)) return IFA_E_INVALID;
    for (uint32_t j = 0; j < n_queries; j++)
        if (!seq[j] || len[j] == 0 || len[j] > IFA_MAX_QUERY_LEN || !clean_name(names[j]))
            return IFA_E_INVALID;
    ifa_sam *w = new (std::nothrow) ifa_sam();
    if (!w) return IFA_E_NOMEM;
    try {
        w->policy = n_policy;
        w->qname.reserve(n_queries);
        w->fwd.reserve(n_queries);
        w->rev.reserve(n_queries);
        for (uint32_t j = 0; j < n_queries; j++) {
            w->qname.emplace_back(names[j]);
            std::string f(len[j], 'N'), r(len[j], 'N');
            for (uint32_t i = 0; i < len[j]; i++) f[i] = norm_base(seq[j][i]);
            for (uint32_t i = 0; i < len[j]; i++) r[i] = comp_base(f[len[j] - 1 - i]);
            w->fwd.push_back(std::move(f));
            w->rev.push_back(std::move(r));
        }
        w->seen.assign(n_queries, 0);
    } catch (const std::bad_alloc &) {
        delete w;
        return IFA_E_NOMEM;
    }
    *out = w;
    return IFA_OK;
}

void ifa_sam_destroy(ifa_sam *w) { delete w; }

const char *ifa_sam_last_error(const ifa_sam *w) { return w ? w->err.c_str() : ""; }

ifa_status ifa_sam_add_contigs(ifa_sam *w, uint32_t first_ordinal, uint32_t n,
                               const char *const *names, const uint64_t *len)
{
    if (!w) return IFA_E_INVALID;
    w->err.clear();
    if (first_ordinal != w->cname.size()) {
        w->err = "contigs must be added in ordinal order: expected ordinal " +
                 std::to_string(w->cname.size());
        return IFA_E_INVALID;
    }
    if (n > 0 && (!names || !len)) {
        w->err = "NULL argument";
        return IFA_E_INVALID;
    }
    for (uint32_t i = 0; i < n; i++)
        if (!clean_name(names[i]) || len[i] >= (1ull << 31)) {
            w->err = "contig " + std::to_string(first_ordinal + i) +
                     ": empty name, tab or newline in it, or length >= 2^31";
            return IFA_E_INVALID;
        }
    try {
        for (uint32_t i = 0; i < n; i++) {
            w->cname.emplace_back(names[i]);
            w->clen.push_back(len[i]);
        }
    } catch (const std::bad_alloc &) {
        w->cname.resize(first_ordinal);
        w->clen.resize(first_ordinal);
        return IFA_E_NOMEM;
    }
    return IFA_OK;
}

ifa_status ifa_sam_header(const ifa_sam *w, char *buf, uint64_t cap, uint64_t *n_bytes)
{
    if (!w || !n_bytes) return IFA_E_INVALID;
    std::string h;
    try {
        h = "@HD\tVN:1.6\tSO:coordinate\n";
        for (size_t i = 0; i < w->cname.size(); i++) {
            h += "@SQ\tSN:";
            h += w->cname[i];
            h += "\tLN:";
            put_u64(h, w->clen[i]);
            h += '\n';
        }
        h += "@PG\tID:ifa\tPN:ifa\tVN:";
        put_u64(h, IFA_ABI_VERSION);
        h += '\n';
    } catch (const std::bad_alloc &) {
        return IFA_E_NOMEM;
    }
    *n_bytes = h.size();
    if (!buf) return IFA_OK;
    if (cap < h.size()) return IFA_E_INVALID;
    std::memcpy(buf, h.data(), h.size());
    return IFA_OK;
}

ifa_status ifa_sam_format(ifa_sam *w, const ifa_hit *hits, uint64_t n, char *buf, uint64_t cap,
                          uint64_t *n_consumed, uint64_t *n_bytes)
{
    if (!w || !n_consumed || !n_bytes || (n > 0 && (!hits || !buf))) return IFA_E_INVALID;
    w->err.clear();
    *n_consumed = 0;
    *n_bytes = 0;
    try {
        return format_hits(w, hits, n, buf, cap, n_consumed, n_bytes);
    } catch (const std::bad_alloc &) {
        return IFA_E_NOMEM;
    }
}

}  // extern "C"

static ifa_status format_hits(ifa_sam *w, const ifa_hit *hits, uint64_t n, char *buf,
                              uint64_t cap, uint64_t *n_consumed, uint64_t *n_bytes)
{
    std::string line;
    uint64_t used = 0;
    for (uint64_t i = 0; i < n; i++) {
        const ifa_hit &h = hits[i];
        if (h.query >= w->fwd.size()) {
            w->err = "hit " + std::to_string(i) + ": query index out of range";
            return i ? IFA_OK : IFA_E_INVALID;
        }
        if (h.contig >= w->cname.size()) {
            w->err = "hit " + std::to_string(i) + ": contig ordinal " + std::to_string(h.contig) +
                     " has no name (ifa_sam_add_contigs)";
            return i ? IFA_OK : IFA_E_INVALID;
        }
        if (w->have_last && before(h, w->last)) {
            w->err = "hit " + std::to_string(i) + " is before the previous one in reference order";
            return i ? IFA_OK : IFA_E_INVALID;
        }
        const std::string &s = h.strand ? w->rev[h.query] : w->fwd[h.query];
        const int64_t L = (int64_t)s.size();
        const int64_t cn = (int64_t)w->clen[h.contig];
        const int64_t p = h.pos;
        const int64_t a = p < 0 ? -p : 0;
        const int64_t b = p + L > cn ? p + L - cn : 0;
        if (a + b >= L || h.strand > 1) {
            w->err = "hit " + std::to_string(i) + " does not fit its contig";
            return i ? IFA_OK : IFA_E_INVALID;
        }
        line.clear();
        line += w->qname[h.query];
        line += '\t';
        put_u64(line, (h.strand ? 16u : 0u) | (w->seen[h.query] ? 256u : 0u));
        line += '\t';
        line += w->cname[h.contig];
        line += '\t';
        put_i64(line, (p > 0 ? p : 0) + 1);
        line += "\t255\t";
        if (a) {
            put_i64(line, a);
            line += 'S';
        }
        put_i64(line, L - a - b);
        line += 'M';
        if (b) {
            put_i64(line, b);
            line += 'S';
        }
        line += "\t*\t0\t0\t";
        line += s;
        line += "\t*\tNM:i:";
        const int64_t m = h.mismatches;
        put_i64(line, w->policy == IFA_N_AS_MISMATCH ? m - (a + b) : m);
        line += "\tXN:i:";
        put_i64(line, (int64_t)h.n_ref - (a + b));
        line += '\n';
        if (used + line.size() > cap) {
            if (i == 0) {
                w->err = "buffer too small for one line (" + std::to_string(line.size()) +
                         " bytes)";
                return IFA_E_INVALID;
            }
            break;
        }
        std::memcpy(buf + used, line.data(), line.size());
        used += line.size();
        w->seen[h.query] = 1;
        w->last = h;
        w->have_last = true;
        *n_consumed = i + 1;
        *n_bytes = used;
    }
    return IFA_OK;
}
