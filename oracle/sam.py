"""SAM text for hit records -- TEST INFRASTRUCTURE ONLY (part of the oracle).

Only tests/ may use this module. It writes, plainly and slowly, the SAM text
the library's native writer must produce byte for byte.

What it follows (Methods, "Output Format"): the aligner streams the reference,
so its SAM output is headerless and a separate header (the paper's outh= file)
is concatenated in front of it. Results, "Accuracy Validation": the primary
alignment of a query is the first valid alignment in reference order; every
other alignment of that query is secondary; queries without a hit are not
reported. Readings where the paper is silent (SAM v1.6 field meanings):
  * one line per hit, in the order given (reference order: contig, pos,
    strand, query);
  * FLAG = 16 for the reverse-complement strand, | 256 for a secondary line;
  * RNAME = the contig's name; POS = 1-based first aligned (non-clipped) base;
  * MAPQ = 255 (not available);
  * CIGAR = [aS] (L - a - b)M [bS] in reference orientation, a and b the bases
    that hang off the contig's left and right ends (overhang windows);
  * RNEXT *, PNEXT 0, TLEN 0; SEQ = the strand sequence as compared (the
    query, or its reverse complement), upper case, non-ACGT bytes as N;
    QUAL *;
  * tags NM:i = mismatches over the aligned bases (the record's count; under
    the N-as-mismatch policy without the clipped bases, which it counts too)
    and XN:i = reference Ns over the aligned bases (the record's n_ref without
    the clipped bases, which read as N);
  * header: @HD VN:1.6 SO:coordinate, one @SQ SN/LN line per contig in
    ordinal order, and @PG ID:ifa PN:ifa VN:<ABI version>.
"""
from __future__ import annotations

N_SEPARATE, N_AS_MISMATCH = 0, 1
ABI_VERSION = 4

_NORM = {ord(c): c for c in "ACGT"}
_NORM.update({ord(c.lower()): c for c in "ACGT"})
_COMP = {"A": "T", "C": "G", "G": "C", "T": "A", "N": "N"}


def normalise(seq: bytes) -> str:
    return "".join(_NORM.get(b, "N") for b in seq)


def revcomp(s: str) -> str:
    return "".join(_COMP[c] for c in reversed(s))


def header(contig_names, contig_lens) -> str:
    lines = ["@HD\tVN:1.6\tSO:coordinate"]
    for name, n in zip(contig_names, contig_lens):
        lines.append(f"@SQ\tSN:{name}\tLN:{int(n)}")
    lines.append(f"@PG\tID:ifa\tPN:ifa\tVN:{ABI_VERSION}")
    return "".join(line + "\n" for line in lines)


class SamText:
    """Formats hits; remembers which queries already had their primary line."""

    def __init__(self, queries, query_names, n_policy=N_SEPARATE):
        self.seq = [normalise(bytes(q)) for q in queries]
        self.names = list(query_names)
        self.policy = n_policy
        self.seen = set()

    def lines(self, hits, contig_names, contig_lens) -> str:
        out = []
        for h in hits.tolist():
            q, contig, pos, strand, n_ref, m = (int(x) for x in h)
            s = self.seq[q]
            L = len(s)
            n = int(contig_lens[contig])
            a = max(0, -pos)                    # bases before the contig start
            b = max(0, pos + L - n)             # bases past the contig end
            cigar = (f"{a}S" if a else "") + f"{L - a - b}M" + (f"{b}S" if b else "")
            flag = 16 if strand == 1 else 0
            if q in self.seen:
                flag |= 256
            self.seen.add(q)
            nm = m - (a + b) if self.policy == N_AS_MISMATCH else m
            xn = n_ref - (a + b)
            seq = s if strand == 0 else revcomp(s)
            out.append("\t".join([self.names[q], str(flag), contig_names[contig],
                                  str(max(pos, 0) + 1), "255", cigar, "*", "0", "0", seq, "*",
                                  f"NM:i:{nm}", f"XN:i:{xn}"]) + "\n")
        return "".join(out)
