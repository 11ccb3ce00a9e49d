"""Pins for the oracle's SAM writer (Methods, "Output Format": headerless SAM
plus a separate header; Results, "Accuracy Validation": the primary is the
first valid alignment in reference order, the others are secondary).

Each SAM line is read back with a parser written here from the SAM v1.6
field definitions and checked against the scan by another route: the window
the line implies (POS, CIGAR) is re-evaluated with the oracle's single-window
test and with a direct recount over the contig bytes; SEQ against
bytes.translate reverse complements; FLAG 256 against a first-occurrence rule;
the order against SO:coordinate; the header against the contig table.
"""
import random
import re

import numpy as np
import pytest

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")
CIGAR = re.compile(r"^(?:(\d+)S)?(\d+)M(?:(\d+)S)?$")


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def upper_n(b: bytes) -> bytes:
    return bytes(c if c in b"ACGT" else ord("N") for c in b.upper())


def parse(text):
    rows = []
    for line in text.splitlines():
        f = line.split("\t")
        assert len(f) == 13, line
        m = CIGAR.match(f[5])
        assert m, f[5]
        a, mm, b = (int(x) if x else 0 for x in m.groups())
        assert f[11].startswith("NM:i:") and f[12].startswith("XN:i:")
        rows.append(dict(qname=f[0], flag=int(f[1]), rname=f[2], pos=int(f[3]),
                         mapq=int(f[4]), clip_l=a, match=mm, clip_r=b, rnext=f[6],
                         pnext=int(f[7]), tlen=int(f[8]), seq=f[9], qual=f[10],
                         nm=int(f[11][5:]), xn=int(f[12][5:])))
    return rows


def _case(rng, oracle_mod, policy, overhang):
    qs = [rand_dna(rng, rng.randint(4, 40), b"ACGT" if rng.random() < 0.8 else b"ACGTNacgt")
          for _ in range(rng.randint(1, 5))]
    contigs = [rand_dna(rng, rng.randint(0, 120), rng.choice([b"ACGT", b"ACGTN"]))
               for _ in range(rng.randint(1, 6))]
    for c in range(len(contigs)):                       # planted copies at both ends
        q = rng.choice(qs)
        if len(contigs[c]) > 2 * len(q):
            o = rng.randint(0, len(q) // 4)
            contigs[c] = q[o:] + contigs[c][len(q):-len(q)] + q[:len(q) - o]
    ks = [rng.randint(0, len(q) // 2) for q in qs]
    hits = oracle_mod.scan(qs, contigs, ks, policy=policy, overhang=overhang)
    return qs, contigs, ks, hits


@pytest.mark.parametrize("policy,overhang", [(0, False), (0, True), (1, True)])
def test_sam_lines_read_back_to_their_windows(oracle_mod, policy, overhang):
    from oracle import sam
    rng = random.Random(300 + 2 * policy + overhang)
    checked = 0
    for trial in range(150):
        qs, contigs, ks, hits = _case(rng, oracle_mod, policy, overhang)
        qnames = [f"q{j}" for j in range(len(qs))]
        cnames = [f"chr{c}" for c in range(len(contigs))]
        lens = [len(c) for c in contigs]
        text = sam.SamText(qs, qnames, policy).lines(hits, cnames, lens)
        rows = parse(text)
        assert len(rows) == len(hits)
        first_seen = set()
        last = (-1, 0)
        for r in rows:
            j = qnames.index(r["qname"])
            ci = cnames.index(r["rname"])
            q, c, L = qs[j], contigs[ci], len(qs[j])
            strand = 1 if r["flag"] & 16 else 0
            assert r["flag"] & ~(16 | 256) == 0
            assert (r["mapq"], r["rnext"], r["pnext"], r["tlen"], r["qual"]) == (255, "*", 0, 0, "*")
            # SEQ: the strand sequence, upper case, N for non-ACGT
            want_seq = upper_n(q) if strand == 0 else upper_n(q).translate(COMP)[::-1]
            assert r["seq"].encode() == want_seq
            assert r["clip_l"] + r["match"] + r["clip_r"] == L == len(r["seq"])
            # clips only where the window leaves the contig
            p = r["pos"] - 1 - r["clip_l"]
            assert r["clip_l"] == max(0, -p) and r["clip_r"] == max(0, p + L - len(c))
            assert r["pos"] >= 1 and r["pos"] - 1 + r["match"] <= len(c)
            # recount over the aligned bases, straight from the contig bytes
            ref = upper_n(c[r["pos"] - 1:r["pos"] - 1 + r["match"]])
            seg = r["seq"].encode()[r["clip_l"]:r["clip_l"] + r["match"]]
            if policy == 0:
                nm = sum(1 for x, y in zip(ref, seg) if x != ord("N") and x != y)
            else:
                nm = sum(1 for x, y in zip(ref, seg) if x == ord("N") or y == ord("N") or x != y)
            assert r["nm"] == nm and r["xn"] == ref.count(b"N")
            # the implied window is a hit of the scan with these counts
            ev = oracle_mod.eval_window(q, ks[j], c, p, strand, policy=policy, overhang=overhang)
            assert ev is not None and ev[0]
            clipped = r["clip_l"] + r["clip_r"]
            assert ev[2] == r["xn"] + clipped
            assert ev[1] == r["nm"] + (clipped if policy == 1 else 0)
            # primary: the query's first line in reference order
            assert bool(r["flag"] & 256) == (j in first_seen)
            first_seen.add(j)
            # SO:coordinate: contig in header order, then POS
            assert (ci, r["pos"]) >= last
            last = (ci, r["pos"])
            checked += 1
        # queries without a hit are not reported
        assert first_seen == set(int(x) for x in np.unique(hits["query"]))
    assert checked > 500


def test_primary_state_carries_across_calls(oracle_mod):
    """Splitting the hits over several calls changes no byte: a query's
    primary stays its first line in reference order."""
    from oracle import sam
    rng = random.Random(11)
    qs, contigs, ks, hits = _case(rng, oracle_mod, 0, True)
    while len(hits) < 10:
        qs, contigs, ks, hits = _case(rng, oracle_mod, 0, True)
    names, cn, lens = [f"r{j}" for j in range(len(qs))], [f"c{i}" for i in range(len(contigs))], \
        [len(c) for c in contigs]
    whole = sam.SamText(qs, names).lines(hits, cn, lens)
    w = sam.SamText(qs, names)
    parts = "".join(w.lines(hits[i:i + 3], cn, lens) for i in range(0, len(hits), 3))
    assert parts == whole


def test_header_lists_every_contig_in_order():
    from oracle import sam
    text = sam.header(["a", "chr2", "x y"], [5, 0, 1000])
    lines = text.splitlines()
    assert lines[0].split("\t") == ["@HD", "VN:1.6", "SO:coordinate"]
    sq = [ln.split("\t") for ln in lines if ln.startswith("@SQ")]
    assert [(f[1], f[2]) for f in sq] == [("SN:a", "LN:5"), ("SN:chr2", "LN:0"), ("SN:x y", "LN:1000")]
    assert lines[-1].startswith("@PG\tID:ifa")
    assert text.endswith("\n")
