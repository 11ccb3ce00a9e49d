"""Pins for the oracle: each test checks it against something other than its own
code -- a library routine, a closed form, an invariant of the method, planted
copies of known mismatch count, published generator outputs or a brute force
over tiny inputs.

Method passages: brute-force mode tests every start position and reports every
valid alignment (Methods, "Algorithm Design"); Hamming distance with a
threshold up to the full query length (Abstract; "Mismatch Tolerance
Scalability"); reference Ns tracked apart from substitutions (Methods,
"Algorithm Design"; "SIMD Optimization"); lanes stop when a count exceeds its
threshold ("SIMD Optimization"); 0% false negatives for substitution counts
0-16 ("Accuracy Validation", Table 6).
"""
import os
import random

import numpy as np
import pytest
from scipy.spatial.distance import hamming
from scipy.stats import binom

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")


def revcomp(s: bytes) -> bytes:
    return s.translate(COMP)[::-1]


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def as_set(h):
    return {tuple(int(x) for x in r) for r in h.tolist()}


# ---------------------------------------------------------------------------
# generator / digest mixing: published SplitMix64 outputs
# ---------------------------------------------------------------------------

# SplitMix64 reference outputs for seed 1234567 (the published sequence from
# the reference implementation of Steele, Lea & Flood's generator), kept as a
# fixture with its citation.
_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                       "splitmix64_seed1234567.txt")
with open(_GOLDEN) as _f:
    SPLITMIX64_1234567 = [int(x) for x in _f.read().split("\n") if x and not x.startswith("#")]
assert len(SPLITMIX64_1234567) == 5


def test_splitmix64_published_outputs(synth_mod):
    assert [int(x) for x in synth_mod.splitmix64(1234567, 5)] == SPLITMIX64_1234567


def test_oracle_mix64_is_splitmix_finaliser(oracle_mod):
    # output k of SplitMix64 is the finaliser applied to seed + (k+1) * gamma
    gamma = 0x9E3779B97F4A7C15
    for k, want in enumerate(SPLITMIX64_1234567):
        assert oracle_mod.mix64((1234567 + (k + 1) * gamma) % 2**64) == want


# ---------------------------------------------------------------------------
# brute force over tiny random inputs
# ---------------------------------------------------------------------------

def _rand_case(rng):
    nc = rng.randint(0, 4)
    contigs = []
    for _ in range(nc):
        n = rng.choice([0, 1, 2, 5, 17, 40, 90, 200])
        alpha = rng.choice([b"ACGT", b"ACGTN", b"ACGTNNNN", b"acgtACGTRYN-."])
        contigs.append(rand_dna(rng, n, alpha))
    nq = rng.randint(1, 4)
    qs = []
    for _ in range(nq):
        L = rng.randint(1, 40)
        alpha = b"ACGT" if rng.random() < 0.8 else b"ACGTN"
        qs.append(rand_dna(rng, L, alpha))
    ks = [rng.randint(0, len(q) + 2) for q in qs]
    mn = None if rng.random() < 0.5 else [rng.randint(0, len(q) + 1) for q in qs]
    return qs, contigs, ks, mn


@pytest.mark.parametrize("policy", [0, 1])
def test_oracle_equals_numpy_brute_force(oracle_mod, policy):
    rng = random.Random(12345 + policy)
    for trial in range(1500):
        qs, contigs, ks, mn = _rand_case(rng)
        strands = rng.choice([1, 2, 3, 3, 3])
        a = oracle_mod.scan(qs, contigs, ks, mn, strands=strands, policy=policy,
                            threads=rng.choice([1, 3]))
        b = oracle_mod.brute_scan(qs, contigs, ks, mn, strands=strands, policy=policy)
        assert np.array_equal(a, b), (trial, qs, contigs, ks, mn, strands)


# ---------------------------------------------------------------------------
# special cases that reduce to library routines
# ---------------------------------------------------------------------------

def _find_all(hay: bytes, needle: bytes):
    out, i = [], hay.find(needle)
    while i >= 0:
        out.append(i)
        i = hay.find(needle, i + 1)
    return out


def test_k0_is_exact_matching(oracle_mod):
    """maxSubs = 0 on N-free contigs: hits are exactly the (overlapping)
    occurrences of q (strand +) and of its reverse complement (strand -)."""
    rng = random.Random(7)
    for trial in range(200):
        L = rng.randint(1, 12)
        q = rand_dna(rng, L)
        contigs = []
        for _ in range(rng.randint(1, 3)):
            parts = [rand_dna(rng, rng.randint(0, 60))]
            for _ in range(rng.randint(0, 4)):
                parts.append(rng.choice([q, revcomp(q)]))
                parts.append(rand_dna(rng, rng.randint(0, 20)))
            contigs.append(b"".join(parts))
        h = oracle_mod.scan([q], contigs, [0])
        want = set()
        for ci, c in enumerate(contigs):
            for p in _find_all(c, q):
                want.add((0, ci, p, 0, 0, 0))
            for p in _find_all(c, revcomp(q)):
                want.add((0, ci, p, 1, 0, 0))
        assert as_set(h) == want, trial


def test_mismatch_count_is_scipy_hamming(oracle_mod):
    """maxSubs = L on N-free contigs: every window is reported, and its
    mismatch count is the Hamming distance from scipy."""
    rng = random.Random(11)
    for trial in range(40):
        L = rng.randint(1, 30)
        q = rand_dna(rng, L)
        c = rand_dna(rng, rng.randint(L, 300))
        h = oracle_mod.scan([q], [c], [L], [L])
        qa = np.frombuffer(q, np.uint8)
        qr = np.frombuffer(revcomp(q), np.uint8)
        ca = np.frombuffer(c, np.uint8)
        assert len(h) == 2 * (len(c) - L + 1)
        for row in h:
            w = ca[row["pos"]:row["pos"] + L]
            ref_q = qa if row["strand"] == 0 else qr
            assert row["mismatches"] == round(hamming(ref_q, w) * L)
            assert row["n_ref"] == 0


@pytest.mark.parametrize("strands,mult", [(1, 1), (2, 1), (3, 2)])
def test_full_threshold_closed_form(oracle_mod, strands, mult):
    """maxSubs = maxN = L: every in-contig window is a hit, so each query has
    strands * sum_c max(0, n_c - L + 1) hits (Ns included)."""
    rng = random.Random(3)
    contigs = [rand_dna(rng, n, b"ACGTN") for n in (0, 3, 10, 57, 130)]
    qs = [rand_dna(rng, L) for L in (1, 4, 10, 11, 60)]
    h = oracle_mod.scan(qs, contigs, [len(q) for q in qs], [len(q) for q in qs],
                        strands=strands)
    for j, q in enumerate(qs):
        want = mult * sum(max(0, len(c) - len(q) + 1) for c in contigs)
        assert int((h["query"] == j).sum()) == want


# ---------------------------------------------------------------------------
# planted copies of known mismatch count (Table 6 protocol)
# ---------------------------------------------------------------------------

def test_planted_c1_recall(oracle_mod, synth_mod):
    w = synth_mod.c1_tiny()
    h = oracle_mod.scan(w.queries, w.ref, w.max_subs)
    got = as_set(h)
    for p in w.plants:
        assert (p.query, p.contig, p.pos, p.strand, 0, p.subs) in got
    # no window other than the planted ones reaches 3 mismatches at L = 32
    assert len(h) == len(w.plants) == 20


def _mutate(rng, q: bytes, s: int):
    a = bytearray(q)
    where = rng.sample(range(len(q)), s)
    for i in where:
        a[i] = rng.choice([b for b in b"ACGT" if b != a[i]])
    return bytes(a), set(where)


@pytest.mark.parametrize("policy", [0, 1])
def test_planted_with_reference_ns(oracle_mod, policy):
    """A copy with s substitutions and t reference Ns at other positions:
    N_SEPARATE reports m = s, n_ref = t and needs t <= maxN;
    N_AS_MISMATCH reports m = s + t and has no maxN test."""
    rng = random.Random(21 + policy)
    for trial in range(300):
        L = rng.randint(4, 40)
        q = rand_dna(rng, L)
        s = rng.randint(0, L // 3)
        t = rng.randint(0, L // 3)
        copy, subs_at = _mutate(rng, q, s)
        free = [i for i in range(L) if i not in subs_at]
        n_at = rng.sample(free, min(t, len(free)))
        t = len(n_at)
        a = bytearray(copy)
        for i in n_at:
            a[i] = ord("N")
        strand = rng.randint(0, 1)
        win = bytes(a) if strand == 0 else revcomp(bytes(a)).replace(b"N", b"N")
        left, right = rand_dna(rng, 5), rand_dna(rng, 5)
        contig = left + win + right
        k = rng.randint(0, L)
        maxn = rng.randint(0, L)
        h = oracle_mod.scan([q], [contig], [k], [maxn], strands=1 << strand, policy=policy)
        rows = [r for r in h.tolist() if r[2] == 5]
        if policy == 0:
            expect_hit = s <= k and t <= maxn
            expect = (0, 0, 5, strand, t, s)
        else:
            expect_hit = s + t <= k
            expect = (0, 0, 5, strand, t, s + t)
        assert (expect in {tuple(r) for r in rows}) == expect_hit, (trial, L, s, t, k, maxn)
        if not expect_hit:
            assert rows == []


def test_threshold_is_inclusive_and_default_maxn_is_floor_quarter(oracle_mod):
    rng = random.Random(5)
    for L in range(1, 41):
        q = rand_dna(rng, L)
        for s in range(0, min(L, 6) + 1):
            copy, _ = _mutate(rng, q, s)
            h = oracle_mod.scan([q], [copy], [s], strands=1)
            assert as_set(h) == {(0, 0, 0, 0, 0, s)}
            if s > 0:
                assert len(oracle_mod.scan([q], [copy], [s - 1], strands=1)) == 0
        # t Ns and no substitutions; default maxN = floor(L / 4)
        for t in range(0, L + 1):
            a = bytearray(q)
            for i in rng.sample(range(L), t):
                a[i] = ord("N")
            h = oracle_mod.scan([q], [bytes(a)], [0], strands=1)
            assert (len(h) == 1) == (t <= L // 4), (L, t)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_reverse_complement_symmetry(oracle_mod):
    """Scanning RC(contig) maps a hit at (p, strand) to (n - L - p, 1 - strand)
    with the same counts; scanning RC(q) swaps the strands."""
    rng = random.Random(9)
    for trial in range(150):
        L = rng.randint(1, 15)
        q = rand_dna(rng, L, b"ACGTN" if trial % 5 == 0 else b"ACGT")
        c = rand_dna(rng, rng.randint(0, 120), b"ACGTN" if trial % 3 == 0 else b"ACGT")
        k = rng.randint(0, L)
        h1 = as_set(oracle_mod.scan([q], [c], [k], [L]))
        h2 = as_set(oracle_mod.scan([q], [revcomp(c)], [k], [L]))
        n = len(c)
        mapped = {(j, ci, n - L - p, 1 - s, nr, m) for (j, ci, p, s, nr, m) in h1}
        assert mapped == h2, trial
        h3 = as_set(oracle_mod.scan([revcomp(q)], [c], [k], [L]))
        assert {(j, ci, p, 1 - s, nr, m) for (j, ci, p, s, nr, m) in h1} == h3


def test_monotone_in_threshold(oracle_mod):
    rng = random.Random(13)
    q = [rand_dna(rng, 14), rand_dna(rng, 9)]
    cs = [rand_dna(rng, 400, b"ACGTN"), rand_dna(rng, 300)]
    prev = None
    for k in range(0, 15):
        cur = as_set(oracle_mod.scan(q, cs, [k, k]))
        if prev is not None:
            assert prev <= cur
            assert {r for r in cur if r[5] <= k - 1} == prev
        prev = cur


def test_contig_ordinals_and_split_calls(oracle_mod):
    rng = random.Random(17)
    q = [rand_dna(rng, 6), rand_dna(rng, 8)]
    cs = [rand_dna(rng, rng.randint(0, 200), b"ACGTN") for _ in range(6)]
    whole = as_set(oracle_mod.scan(q, cs, [2, 3]))
    parts = set()
    for i, c in enumerate(cs):
        parts |= as_set(oracle_mod.scan(q, [c], [2, 3], first_ordinal=i))
    assert whole == parts
    # thread count does not change the result
    assert whole == as_set(oracle_mod.scan(q, cs, [2, 3], threads=7))


def test_palindromic_query_reports_both_strands(oracle_mod):
    q = b"ACGT"        # its own reverse complement
    h = oracle_mod.scan([q], [b"TTACGTTT"], [0])
    assert as_set(h) == {(0, 0, 2, 0, 0, 0), (0, 0, 2, 1, 0, 0)}


def test_duplicate_queries_reported_independently(oracle_mod):
    h = oracle_mod.scan([b"ACG", b"ACG"], [b"ACGA"], [0, 0], strands=1)
    assert as_set(h) == {(0, 0, 0, 0, 0, 0), (1, 0, 0, 0, 0, 0)}


def test_case_insensitive_and_iupac_is_n(oracle_mod):
    q = b"ACGTAC"
    h_up = as_set(oracle_mod.scan([q], [b"GGACGTACGG"], [0], strands=1))
    h_lo = as_set(oracle_mod.scan([q.lower()], [b"ggacgtacgg"], [0], strands=1))
    assert h_up == h_lo == {(0, 0, 2, 0, 0, 0)}
    # R, Y, '-', '.', 'U' are all N: one in the window -> n_ref 1, m 0
    for b in b"RY-.UnX":
        c = b"GGACG" + bytes([b]) + b"ACGG"
        assert as_set(oracle_mod.scan([q], [c], [0], [1], strands=1)) == {(0, 0, 2, 0, 1, 0)}


def test_query_n_rules(oracle_mod):
    # query N against reference A/C/G/T is a substitution
    assert as_set(oracle_mod.scan([b"ANGT"], [b"ACGT"], [1], strands=1)) == {(0, 0, 0, 0, 0, 1)}
    assert len(oracle_mod.scan([b"ANGT"], [b"ACGT"], [0], strands=1)) == 0
    # query N against reference N counts only in n_ref
    assert as_set(oracle_mod.scan([b"ANGT"], [b"ANGT"], [0], [1], strands=1)) == \
        {(0, 0, 0, 0, 1, 0)}


def test_edge_cases(oracle_mod):
    assert len(oracle_mod.scan([b"ACGT"], [], [1])) == 0
    assert len(oracle_mod.scan([b"ACGT"], [b""], [1])) == 0
    assert len(oracle_mod.scan([b"ACGT"], [b"ACG"], [4])) == 0
    # maxSubs above L is clamped to L: every window is a hit
    assert len(oracle_mod.scan([b"AC"], [b"GGGG"], [99], [2], strands=1)) == 3
    # L = 1
    assert as_set(oracle_mod.scan([b"A"], [b"CAT"], [0], strands=3)) == \
        {(0, 0, 1, 0, 0, 0), (0, 0, 2, 1, 0, 0)}
    with pytest.raises(ValueError):
        oracle_mod.scan([b"ACGT"], [b"ACGT"], [-1])


def test_eval_window_agrees_with_scan(oracle_mod):
    rng = random.Random(23)
    for _ in range(100):
        L = rng.randint(1, 20)
        q = rand_dna(rng, L, b"ACGTN")
        c = rand_dna(rng, rng.randint(L, 80), b"ACGTN")
        k = rng.randint(0, L)
        hits = as_set(oracle_mod.scan([q], [c], [k]))
        for p in range(len(c) - L + 1):
            for s in (0, 1):
                ok, m, nr = oracle_mod.eval_window(q, k, c, p, s)
                assert ok == ((0, 0, p, s, nr, m) in hits)


# ---------------------------------------------------------------------------
# statistics of random hits (not exact; wide bound)
# ---------------------------------------------------------------------------

def test_random_hit_rate_matches_binomial(oracle_mod, synth_mod):
    """With iid uniform queries a base matches with probability 1/4 whatever
    the reference composition, so the expected hit count is
    strands * windows * P(Bin(L, 3/4) <= k)."""
    spec = synth_mod.RefSpec(seed=99, length_mode=0, n_fixed=4, fixed_len=100_000,
                             gc_lo=0.5, gc_hi=0.5)
    ref = synth_mod.gen_reference(spec)
    nq = 60
    qs = synth_mod.gen_queries(99, nq, 12, 12)
    k = 3
    h = oracle_mod.scan(qs, ref, [k] * nq)
    W = sum(int(n) - 12 + 1 for n in ref.lens)
    expect = 2 * W * binom.cdf(k, 12, 0.75)          # per query
    per_q = np.bincount(h["query"], minlength=nq).astype(float)
    # overlapping windows make per-query counts over-dispersed; bound the mean
    # by its empirical standard error
    se = per_q.std(ddof=1) / np.sqrt(nq)
    assert abs(per_q.mean() - expect) < 5 * se + 1, (per_q.mean(), expect, se)
    # a wrong threshold (k - 1 or k + 1) would move the mean far outside that bound
    for wrong in (k - 1, k + 1):
        assert abs(2 * W * binom.cdf(wrong, 12, 0.75) - expect) > 10 * se


# ---------------------------------------------------------------------------
# count+digest agrees with the records
# ---------------------------------------------------------------------------

def test_count_digest_matches_records(oracle_mod):
    rng = random.Random(29)
    qs = [rand_dna(rng, L) for L in (5, 7, 9)]
    cs = [rand_dna(rng, 500, b"ACGTN") for _ in range(3)]
    h, counts, digests = oracle_mod.scan(qs, cs, [2, 3, 4], stats=True, first_ordinal=40)
    for j in range(3):
        rows = h[h["query"] == j]
        assert counts[j] == len(rows)
        d = 0
        for r in rows:
            d = (d + oracle_mod.hit_hash(int(r["contig"]), int(r["pos"]), int(r["strand"]),
                                         int(r["mismatches"]), int(r["n_ref"]))) % 2**64
        assert int(digests[j]) == d


def test_fixture_digest_of_records_matches_the_oracle_sink(oracle_mod):
    """The helper that reduces records to (count, digest) for the full-size
    fixtures gives the oracle's own count+digest figures (C1 and a random
    case with query Ns and reference N runs)."""
    import os
    import random
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from workload_fixtures import records_digest
    import synth
    w = synth.c1_tiny()
    hits, cnt, dig = oracle_mod.scan(w.queries, w.ref, w.max_subs, stats=True)
    c2, d2 = records_digest(hits, len(w.queries))
    assert np.array_equal(c2, cnt) and np.array_equal(d2, dig)
    rng = random.Random(17)
    qs = [bytes(rng.choice(b"ACGTN") for _ in range(rng.randint(5, 40))) for _ in range(6)]
    contigs = [bytes(rng.choice(b"ACGTNN") for _ in range(3000)) for _ in range(3)]
    ks = [len(q) // 2 for q in qs]
    hits, cnt, dig = oracle_mod.scan(qs, contigs, ks, stats=True, first_ordinal=7)
    assert len(hits) > 100
    c2, d2 = records_digest(hits, len(qs))
    assert np.array_equal(c2, cnt) and np.array_equal(d2, dig)
