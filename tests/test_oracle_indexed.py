"""Pins for the oracle's indexed mode (Methods, "Algorithm Design": multi-K
seeds with an optional masked centre, MinHits by Monte Carlo with a fixed
seed, a deterministic bound validKmers - kEffective x maxSubs - maxClips at
probability 100 %).

Each test checks against something other than the oracle's own code: the
published SplitMix64 outputs, an exact enumeration of every substitution
placement, brute-force seed counting by byte slicing, exact matching by
bytes.find, and invariants of the method (indexed hits are brute-force hits;
raising a threshold only removes hits).
"""
import itertools
import math
import os
import random

import numpy as np
import pytest

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")
HERE = os.path.dirname(os.path.abspath(__file__))


def revcomp(s: bytes) -> bytes:
    return s.translate(COMP)[::-1]


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def as_set(h):
    return {tuple(int(x) for x in r) for r in h.tolist()}


def test_splitmix_stream_is_the_published_sequence(oracle_mod):
    with open(os.path.join(HERE, "golden", "splitmix64_seed1234567.txt")) as f:
        gold = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    assert [oracle_mod.splitmix64(1234567, n) for n in range(len(gold))] == gold


def _unmasked(t, k, mask):
    lo = (k - mask) // 2
    return t < lo or t >= lo + mask


def _exact_tail(V, s, k, mask, step):
    """P(X >= t) for every t, X = seeds with no substitution at an unmasked
    position, over every placement of s distinct substitutions in the span."""
    span = (V - 1) * step + k
    s = min(s, span)
    hist = [0] * (V + 1)
    for subs in itertools.combinations(range(span), s):
        alive = sum(1 for v in range(V)
                    if not any(0 <= x - v * step < k and _unmasked(x - v * step, k, mask)
                               for x in subs))
        hist[alive] += 1
    total = sum(hist)
    tail, acc = [0.0] * (V + 2), 0
    for t in range(V, -1, -1):
        acc += hist[t]
        tail[t] = acc / total
    return tail, hist


def test_minhits_equals_the_exact_quantile(oracle_mod):
    """Where the exact tail probability is clear of the target by six
    standard errors of the trial count, the Monte Carlo answer is the exact
    quantile."""
    iters = 40_000
    checked = 0
    rng = random.Random(3)
    cases = [(V, s, k, mask, step) for V in (3, 6, 10, 16) for s in (1, 2, 3)
             for (k, mask) in ((4, 0), (6, 0), (7, 3)) for step in (1, 2)]
    rng.shuffle(cases)
    for V, s, k, mask, step in cases[:40]:
        if math.comb((V - 1) * step + k, s) > 60_000:
            continue
        tail, _ = _exact_tail(V, s, k, mask, step)
        for P in (0.5, 0.9, 0.99, 0.999):
            want = max(t for t in range(V + 1) if tail[t] >= P)
            margin = 6 * math.sqrt(P * (1 - P) / iters) + 1e-9
            if tail[want] < P + margin or tail[want + 1] > P - margin:
                continue
            got = oracle_mod.minhits(V, s, k, mask, step, iters=iters, seed=7,
                                     ppm=int(round(P * 1e6)))
            assert got == want, (V, s, k, mask, step, P)
            checked += 1
    assert checked >= 25


def test_deterministic_bound_is_a_worst_case_bound(oracle_mod):
    """At probability 100 %: V - kEffective * maxSubs never exceeds the
    fewest seeds any placement leaves, and kEffective is the most seeds one
    substitution can touch (found by trying every position)."""
    for V, s, k, mask, step in itertools.product((2, 5, 9), (0, 1, 2, 3), (4, 5, 7), (0, 2),
                                                 (1, 2, 3)):
        if mask >= k or math.comb((V - 1) * step + k, s) > 20_000:
            continue
        tail, hist = _exact_tail(V, s, k, mask, step)
        worst = min(t for t in range(V + 1) if hist[t])
        b = oracle_mod.minhits(V, s, k, mask, step, ppm=1_000_000)
        assert b <= worst, (V, s, k, mask, step)
        span = (V - 1) * step + k
        touch = max(sum(1 for v in range(V) if 0 <= x - v * step < k
                        and _unmasked(x - v * step, k, mask)) for x in range(span))
        assert oracle_mod.keff(k, mask, step) >= touch
        if V * step >= k:          # some position is covered by the full pattern
            assert oracle_mod.keff(k, mask, step) == touch
        if s == 0:
            assert b == V


def _py_seed_hits(q: bytes, w: bytes, k, mask, step):
    lo = (k - mask) // 2
    keep = [t for t in range(k) if t < lo or t >= lo + mask]
    up_q, up_w = q.upper(), w.upper()
    n = 0
    for i in range(0, len(q) - k + 1, step):
        qs = bytes(up_q[i + t] for t in keep)
        ws = bytes(up_w[i + t] for t in keep)
        if all(c in b"ACGT" for c in qs) and qs == ws:
            n += 1
    return n


@pytest.mark.parametrize("mask,step", [(0, 1), (2, 1), (0, 2), (3, 3)])
def test_seed_condition_against_byte_slicing(oracle_mod, mask, step):
    rng = random.Random(50 + 7 * mask + step)
    for trial in range(120):
        qs = [rand_dna(rng, rng.randint(6, 30), b"ACGT" if rng.random() < 0.8 else b"ACGTN")
              for _ in range(rng.randint(1, 3))]
        contigs = [rand_dna(rng, rng.randint(0, 80), b"ACGT" if rng.random() < 0.7 else b"ACGTN")
                   for _ in range(rng.randint(1, 3))]
        for c in range(len(contigs)):         # plant near copies so seeds match
            q = rng.choice(qs)
            if len(contigs[c]) >= len(q):
                p = rng.randint(0, len(contigs[c]) - len(q))
                src = q if rng.random() < 0.5 else revcomp(q)
                contigs[c] = contigs[c][:p] + src + contigs[c][p + len(q):]
        ks = [rng.randint(max(mask + 1, 3), min(len(q), 10)) for q in qs]
        thr = [[rng.randint(1, 3), rng.randint(1, 3)] for _ in qs]
        seeds = {"k": ks, "thr": thr, "mask": mask, "step": step}
        L_all = [len(q) for q in qs]
        got = as_set(oracle_mod.scan(qs, contigs, L_all, L_all, seeds=seeds, threads=1))
        want = set()
        for j, q in enumerate(qs):
            L = len(q)
            for ci, c in enumerate(contigs):
                for p in range(0, len(c) - L + 1):
                    w = c[p:p + L]
                    for s, strand in ((0, q), (1, revcomp(q))):
                        if _py_seed_hits(strand, w, ks[j], mask, step) >= thr[j][s]:
                            want.add((j, ci, p, s))
        assert {r[:4] for r in got} == want, trial


def test_all_seeds_required_is_exact_matching(oracle_mod):
    """Step 1, no mask, threshold = every seed of an N-free query: only
    windows equal to the strand sequence qualify (bytes.find), whatever
    maxSubs allows."""
    rng = random.Random(61)
    for trial in range(80):
        L = rng.randint(6, 20)
        q = rand_dna(rng, L, b"AC")
        c = rand_dna(rng, rng.randint(L, 200), b"AC")
        k = rng.randint(2, L)
        V = L - k + 1
        h = oracle_mod.scan([q], [c], [L], [L], seeds={"k": [k], "thr": [[V, V]], "mask": 0,
                                                       "step": 1})
        for s, strand in ((0, q), (1, revcomp(q))):
            pos = {r[2] for r in as_set(h) if r[3] == s}
            want = {i for i in range(len(c) - L + 1) if c[i:i + L] == strand}
            assert pos == want, trial


def test_indexed_hits_are_brute_force_hits_and_monotone(oracle_mod):
    rng = random.Random(71)
    for trial in range(60):
        qs = [rand_dna(rng, rng.randint(12, 40)) for _ in range(3)]
        contigs = [rand_dna(rng, 300) for _ in range(2)]
        for c in range(2):
            q = rng.choice(qs)
            contigs[c] = contigs[c][:100] + q + contigs[c][100 + len(q):]
        ks = [rng.randint(0, 8) for _ in qs]
        brute = as_set(oracle_mod.scan(qs, contigs, ks))
        prev = None
        for t in (1, 2, 4, 8):
            seeds = {"k": [6] * 3, "thr": [[t, t]] * 3, "mask": 0, "step": 1}
            cur = as_set(oracle_mod.scan(qs, contigs, ks, seeds=seeds))
            assert cur <= brute
            if prev is not None:
                assert cur <= prev
            prev = cur


def test_longest_k_rule(oracle_mod):
    """No substitutions: every seed survives, so the longest candidate k that
    fits is chosen and the threshold is the seed count; many substitutions on
    a short query leave no k with MinHits >= 1, so the shortest is taken with
    threshold 1."""
    rng = random.Random(81)
    q = rand_dna(rng, 32)
    p = oracle_mod.indexed_params([q], [0], iters=2000)
    assert p["k"] == [14] and p["thr"] == [[32 - 14 + 1] * 2]
    p = oracle_mod.indexed_params([rand_dna(rng, 20)], [12], iters=2000)
    assert p["k"] == [8] and p["thr"] == [[1, 1]]
    p = oracle_mod.indexed_params([rand_dna(rng, 5)], [0], iters=2000)
    assert p["k"] == [5] and p["thr"] == [[1, 1]]
    # thresholds follow MinHits of each strand's own valid-seed count
    q = b"ACGTACGTNNACGTACGTACGTACGT"
    p = oracle_mod.indexed_params([q], [1], iters=5000)
    k = p["k"][0]
    for s, strand in ((0, q), (1, revcomp(q))):
        lo = k // 2
        v = sum(1 for i in range(len(q) - k + 1) if b"N" not in strand[i:i + k])
        assert p["thr"][0][s] == max(1, oracle_mod.minhits(v, 1, k, iters=5000))
