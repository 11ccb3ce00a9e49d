"""The library's native SAM writer (ifa_sam_*, host code) against the oracle's
SAM text, byte for byte, on hits the oracle found; plus its error paths. No
GPU is needed: the writer does no device work."""
import random

import numpy as np
import pytest

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


@pytest.fixture(scope="module")
def ifa():
    import paper_2607_27291_amd as m
    m.lib()
    return m


def _case(rng, orc, policy, overhang):
    qs = [rand_dna(rng, rng.randint(1, 60), b"ACGT" if rng.random() < 0.8 else b"ACGTNacgtRY")
          for _ in range(rng.randint(1, 6))]
    contigs = [rand_dna(rng, rng.randint(0, 200), rng.choice([b"ACGT", b"ACGTN"]))
               for _ in range(rng.randint(0, 8))]
    for c in range(len(contigs)):
        q = rng.choice(qs)
        if len(contigs[c]) > 2 * len(q):
            o = rng.randint(0, len(q) // 4)
            src = q if rng.random() < 0.5 else q.translate(COMP)[::-1]
            contigs[c] = src[o:] + contigs[c][len(q):-len(q)] + src[:len(q) - o]
    ks = [rng.randint(0, len(q) // 2 + 1) for q in qs]
    return qs, contigs, ks, orc.scan(qs, contigs, ks, policy=policy, overhang=overhang, threads=1)


@pytest.mark.parametrize("policy,overhang", [(0, False), (0, True), (1, True)])
def test_native_sam_equals_oracle_sam(ifa, oracle_mod, policy, overhang):
    from oracle import sam
    rng = random.Random(400 + 2 * policy + overhang)
    lines = 0
    for trial in range(120):
        qs, contigs, ks, hits = _case(rng, oracle_mod, policy, overhang)
        qn = [f"read_{j}/1" for j in range(len(qs))]
        cn = [f"contig {i} x" for i in range(len(contigs))]
        lens = [len(c) for c in contigs]
        want = sam.SamText(qs, qn, policy).lines(hits, cn, lens)
        with ifa.SamWriter(qs, qn, policy) as w:
            # contigs registered over two calls, hits formatted in slices
            cut = rng.randint(0, len(contigs))
            w.add_contigs(cn[:cut], lens[:cut])
            w.add_contigs(cn[cut:], lens[cut:])
            assert w.header() == sam.header(cn, lens)
            got = "".join(w.format(hits[i:i + 7]) for i in range(0, len(hits), 7))
        assert got == want, trial
        lines += want.count("\n")
    assert lines > 300


def test_small_buffers_consume_whole_lines(ifa, oracle_mod):
    from oracle import sam
    rng = random.Random(9)
    qs, contigs, ks, hits = _case(rng, oracle_mod, 0, True)
    while len(hits) < 20:
        qs, contigs, ks, hits = _case(rng, oracle_mod, 0, True)
    qn, cn = [f"q{j}" for j in range(len(qs))], [f"c{i}" for i in range(len(contigs))]
    lens = [len(c) for c in contigs]
    want = sam.SamText(qs, qn).lines(hits, cn, lens)
    longest = max(len(x) + 1 for x in want.splitlines())
    w = ifa.ifa_sam_create(qs, qn)
    try:
        ifa.ifa_sam_add_contigs(w, 0, cn, lens)
        parts, i = [], 0
        while i < len(hits):
            text, used = ifa.ifa_sam_format(w, hits[i:], longest + 5)
            assert used >= 1 and text.endswith("\n")
            parts.append(text)
            i += used
        assert "".join(parts) == want
    finally:
        ifa.ifa_sam_destroy(w)


def test_sam_writer_errors(ifa):
    hit = np.zeros(3, dtype=ifa.HIT_DTYPE)
    with ifa.SamWriter([b"ACGTACGT"], ["q"]) as w:
        w.add_contigs(["c0"], [100])
        with pytest.raises(ifa.IfaError):          # contigs out of ordinal order
            ifa.ifa_sam_add_contigs(w.w, 5, ["c5"], [10])
        with pytest.raises(ifa.IfaError):          # tab in a name
            ifa.ifa_sam_add_contigs(w.w, 1, ["a\tb"], [10])
        hit[0] = (0, 1, 0, 0, 0, 0)                # contig 1 has no name
        with pytest.raises(ifa.IfaError):
            w.format(hit[:1])
        hit[0] = (1, 0, 0, 0, 0, 0)                # query 1 does not exist
        with pytest.raises(ifa.IfaError):
            w.format(hit[:1])
        hit[0] = (0, 0, 95, 0, 0, 0)               # 8-base window at 95 of a 100-base contig
        hit[1] = (0, 0, 10, 0, 0, 0)               # then a hit before it
        text, used = ifa.ifa_sam_format(w.w, hit[:2], 1 << 16)
        assert used == 1 and "\t96\t255\t5M3S\t" in text
        with pytest.raises(ifa.IfaError):
            w.format(hit[1:2])
        hit[2] = (0, 0, 200, 0, 0, 0)              # window off its contig
        with pytest.raises(ifa.IfaError):
            w.format(hit[2:3])
        with pytest.raises(ifa.IfaError):          # buffer shorter than one line
            ifa.ifa_sam_format(w.w, hit[:1], 8)
    with pytest.raises(ifa.IfaError):
        ifa.SamWriter([b"ACGT"], ["bad\nname"])
    with pytest.raises(ifa.IfaError):
        ifa.SamWriter([b""], ["q"])
