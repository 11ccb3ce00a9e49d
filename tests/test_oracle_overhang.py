"""Pins for the oracle's overhang option (soft-clipped windows at contig ends).

Method passages: both modes report alignments that hang off a contig end by up
to 25 % of the query length by default; short contigs are fused with N padding
and the kernel counts reference Ns apart from substitutions (Methods,
"Algorithm Design"; "SIMD Optimization"). Readings: a window may start at
p in [-C, n - L + C] with C = min(maxN, L - 1); off-contig bases read as N;
at most C of a window's bases may be off the contig; pos is the window's first
base (negative for a left overhang).

Each test checks the oracle against something other than its own code: a
numpy brute force over an explicitly N-padded contig, numpy's full-mode
correlation (a library routine), planted copies of known overhang and
mismatch count, closed-form window counts and the reverse-complement
symmetry of the method.
"""
import random

import numpy as np
import pytest

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")


def revcomp(s: bytes) -> bytes:
    return s.translate(COMP)[::-1]


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def as_set(h):
    return {tuple(int(x) for x in r) for r in h.tolist()}


def _rand_case(rng):
    nc = rng.randint(0, 4)
    contigs = []
    for _ in range(nc):
        n = rng.choice([0, 1, 2, 5, 9, 17, 40, 90])
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
def test_overhang_oracle_equals_padded_brute_force(oracle_mod, policy):
    rng = random.Random(777 + policy)
    for trial in range(1200):
        qs, contigs, ks, mn = _rand_case(rng)
        strands = rng.choice([1, 2, 3, 3])
        a = oracle_mod.scan(qs, contigs, ks, mn, strands=strands, policy=policy,
                            overhang=True, threads=rng.choice([1, 3]))
        b = oracle_mod.brute_scan(qs, contigs, ks, mn, strands=strands, policy=policy,
                                  overhang=True)
        assert np.array_equal(a, b), (trial, qs, contigs, ks, mn, strands)


def _onehot(s: bytes):
    a = np.frombuffer(s, dtype=np.uint8)
    return [(a == b).astype(np.int64) for b in b"ACGT"]


def test_full_correlation_of_one_hot_codes(oracle_mod):
    """maxSubs = L and maxN = L - 1 on N-free contigs: C = L - 1, so every
    start p in [-(L - 1), n - 1] is reported (n + L - 1 windows, the length of
    a full-mode correlation), with m = overlap - matches and n_ref = L -
    overlap, where matches come from numpy's full correlation of the one-hot
    base indicators."""
    rng = random.Random(31)
    for trial in range(120):
        L = rng.randint(1, 24)
        n = rng.randint(1, 60)
        q = rand_dna(rng, L)
        c = rand_dna(rng, n)
        for strand in (0, 1):
            h = oracle_mod.scan([q], [c], [L], [L - 1], strands=1 << strand, overhang=True)
            s = q if strand == 0 else revcomp(q)
            matches = sum(np.correlate(cr, qr, mode="full")
                          for cr, qr in zip(_onehot(c), _onehot(s)))
            assert matches.size == n + L - 1 == len(h), (trial, L, n)
            pos = np.arange(-(L - 1), n)
            overlap = np.minimum(pos + L, n) - np.maximum(pos, 0)
            assert np.array_equal(h["pos"], pos)
            assert np.array_equal(h["strand"], np.full(n + L - 1, strand))
            assert np.array_equal(h["n_ref"].astype(np.int64), L - overlap)
            assert np.array_equal(h["mismatches"].astype(np.int64), overlap - matches)


def _mutate(rng, q: bytes, idx, s):
    a = bytearray(q)
    for i in rng.sample(list(idx), s):
        a[i] = rng.choice([b for b in b"ACGT" if b != a[i]])
    return bytes(a)


@pytest.mark.parametrize("policy", [0, 1])
def test_planted_overhanging_copies(oracle_mod, policy):
    """A copy of q (s substitutions in its on-contig part) that hangs o bases
    off the left or right end: reported at pos -o or n - L + o with n_ref = o
    iff o <= floor(L/4) and s <= k (N_SEPARATE), or o <= floor(L/4) and
    s + o <= k (AS_MISMATCH, off-contig bases count as mismatches)."""
    rng = random.Random(41 + policy)
    for trial in range(400):
        L = rng.randint(4, 48)
        q = rand_dna(rng, L)
        o = rng.randint(1, L // 4 + 2)
        if o >= L:
            continue
        side = rng.randint(0, 1)
        strand = rng.randint(0, 1)
        on = range(o, L) if side == 0 else range(0, L - o)
        s = rng.randint(0, min(3, len(on)))
        copy = _mutate(rng, q, on, s)
        body = copy if strand == 0 else revcomp(copy)
        # the window in forward reference coordinates; the off-contig part of
        # the strand sequence maps to the left end for (side 0, strand 0) etc.
        fwd_left_off = (side == 0) == (strand == 0)
        tail = rand_dna(rng, rng.randint(0, 30))
        if fwd_left_off:
            contig = body[o:] + tail
            pos = -o
        else:
            contig = tail + body[:L - o]
            pos = len(contig) - L + o
        k = rng.randint(0, 6)
        h = oracle_mod.scan([q], [contig], [k], strands=1 << strand, policy=policy,
                            overhang=True)
        got = {tuple(r) for r in h.tolist() if r[2] == pos}
        m = s if policy == 0 else s + o
        expect_hit = o <= L // 4 and m <= k
        assert ((0, 0, pos, strand, o, m) in got) == expect_hit, (trial, L, o, s, k, side)
        if not expect_hit:
            assert got == set()
        # without overhang the same window is never reported
        h0 = oracle_mod.scan([q], [contig], [k], strands=1 << strand, policy=policy)
        assert all(r[2] != pos for r in h0.tolist())


def test_contig_shorter_than_the_query(oracle_mod):
    """A contig holding q[a : L - b]: the window at pos -a hangs off both ends
    and is a hit iff a + b <= floor(L/4)."""
    rng = random.Random(53)
    for trial in range(300):
        L = rng.randint(4, 60)
        q = rand_dna(rng, L)
        a = rng.randint(0, L // 4 + 1)
        b = rng.randint(0, L // 4 + 1)
        if a + b >= L:
            continue
        contig = q[a:L - b]
        h = oracle_mod.scan([q], [contig], [0], strands=1, overhang=True)
        got = {tuple(r) for r in h.tolist()}
        expect_hit = a + b <= L // 4
        assert ((0, 0, -a, 0, a + b, 0) in got) == expect_hit, (trial, L, a, b)


def test_window_counts_closed_form(oracle_mod):
    """maxSubs = L under AS_MISMATCH with the default maxN: only the clip limit
    C = floor(L/4) decides, so a contig of n bases yields every start in
    [-C, n - L + C], n - L + 2C + 1 windows per strand, when n >= L - C (a
    contig shorter than L loses L - n bases to the two ends together), and
    none when n < L - C."""
    rng = random.Random(67)
    for trial in range(200):
        L = rng.randint(1, 40)
        C = L // 4
        n = rng.randint(0, 80)
        q = rand_dna(rng, L)
        c = rand_dna(rng, n)
        h = oracle_mod.scan([q], [c], [L], strands=1, overhang=True, policy=1)
        want = n - L + 2 * C + 1 if n >= L - C else 0
        assert len(h) == want, (trial, L, n)
        if want:
            assert np.array_equal(h["pos"], np.arange(-C, n - L + C + 1))


def test_reverse_complement_symmetry_with_overhang(oracle_mod):
    """Scanning RC(contig) maps a hit at (p, strand) to (n - L - p, 1 - strand)
    with the same counts, overhanging windows included."""
    rng = random.Random(79)
    for trial in range(150):
        L = rng.randint(1, 16)
        q = rand_dna(rng, L, b"ACGTN" if trial % 5 == 0 else b"ACGT")
        c = rand_dna(rng, rng.randint(0, 60), b"ACGTN" if trial % 3 == 0 else b"ACGT")
        k = rng.randint(0, L)
        mn = rng.randint(0, L)
        h1 = as_set(oracle_mod.scan([q], [c], [k], [mn], overhang=True))
        h2 = as_set(oracle_mod.scan([q], [revcomp(c)], [k], [mn], overhang=True))
        n = len(c)
        assert {(j, ci, n - L - p, 1 - s, nr, m) for (j, ci, p, s, nr, m) in h1} == h2, trial


def test_overhang_adds_only_overhanging_windows(oracle_mod):
    """The overhang scan is the plain scan plus windows with a base off the
    contig; each added window keeps at least one base on it."""
    rng = random.Random(83)
    for trial in range(200):
        qs, contigs, ks, mn = _rand_case(rng)
        a = as_set(oracle_mod.scan(qs, contigs, ks, mn, overhang=True))
        b = as_set(oracle_mod.scan(qs, contigs, ks, mn))
        assert b <= a
        for (j, ci, p, s, nr, m) in a - b:
            L, n = len(qs[j]), len(contigs[ci])
            assert p < 0 or p + L > n
            assert p + L >= 1 and p <= n - 1


def test_eval_window_agrees_with_overhang_scan(oracle_mod):
    rng = random.Random(97)
    for trial in range(150):
        L = rng.randint(1, 30)
        q = rand_dna(rng, L, b"ACGTN")
        c = rand_dna(rng, rng.randint(0, 50), b"ACGTN")
        k = rng.randint(0, L)
        mn = rng.randint(0, L)
        policy = rng.randint(0, 1)
        hits = as_set(oracle_mod.scan([q], [c], [k], [mn], policy=policy, overhang=True))
        C = min(mn, L - 1)
        n = len(c)
        for p in range(-L - 2, n + 3):
            for s in (0, 1):
                r = oracle_mod.eval_window(q, k, c, p, s, mn, policy, overhang=True)
                off = max(0, -p) + max(0, p + L - n)
                if off > C or off > L - 1 or p + L <= 0 or p >= n:
                    assert r is None, (trial, p, s)
                    continue
                hit, m, nr = r
                assert hit == ((0, 0, p, s, nr, m) in hits), (trial, p, s)
                # without overhang the window is a window of the scan iff it
                # lies wholly inside the contig
                assert (oracle_mod.eval_window(q, k, c, p, s, mn, policy) is None) == (off > 0)


def test_count_digest_with_negative_positions(oracle_mod):
    """Count+digest over overhanging hits equals the count and the wrapping
    sum of the record hashes, pos entering the hash as its 32-bit pattern."""
    rng = random.Random(101)
    qs = [rand_dna(rng, L) for L in (8, 12, 20)]
    contigs = [rand_dna(rng, n) for n in (3, 10, 25, 60)]
    h, cnt, dig = oracle_mod.scan(qs, contigs, [8, 12, 20], overhang=True, stats=True)
    assert (h["pos"] < 0).any()
    for j in range(len(qs)):
        rows = h[h["query"] == j]
        assert cnt[j] == len(rows)
        acc = 0
        for r in rows.tolist():
            acc = (acc + oracle_mod.hit_hash(r[1], r[2], r[3], r[5], r[4])) % (1 << 64)
        assert int(dig[j]) == acc
        # the hash key takes pos modulo 2^32
        for r in rows.tolist():
            if r[2] < 0:
                key = (r[1] << 32) | (r[2] & 0xffffffff)
                aux = r[3] | (r[5] << 1) | (r[4] << 10)
                assert oracle_mod.hit_hash(r[1], r[2], r[3], r[5], r[4]) == \
                    oracle_mod.mix64(key ^ ((aux << 45) & 0xffffffffffffffff))
