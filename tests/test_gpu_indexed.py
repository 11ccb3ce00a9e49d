"""Indexed mode on the GPU (IFA_FLAG_INDEXED) against the oracle: the seed
length and thresholds the library picks for every query equal the oracle's
(same Monte Carlo stream), and the reported windows are bit-exact on all six
record fields, in reference order, and on the count+digest sink. Inputs are
seeded; each test prints its case before touching the GPU.
"""
import random
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

COMP = bytes.maketrans(b"ACGTacgt", b"TGCAtgca")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def revcomp(s: bytes) -> bytes:
    return s.translate(COMP)[::-1]


@pytest.fixture(scope="module")
def ifa():
    import paper_2607_27291_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def assert_same(a, b, ctx=""):
    if not np.array_equal(a, b):
        sa = {tuple(r) for r in a.tolist()}
        sb = {tuple(r) for r in b.tolist()}
        raise AssertionError(f"{ctx}: gpu {len(a)} oracle {len(b)}; only gpu "
                             f"{sorted(sa - sb)[:5]} only oracle {sorted(sb - sa)[:5]}")


def _mutate(rng, q: bytes, s: int) -> bytes:
    a = bytearray(q)
    for i in rng.sample(range(len(q)), min(s, len(q))):
        a[i] = rng.choice([b for b in b"ACGT" if b != a[i]])
    return bytes(a)


def _planted(rng, qs, ks, n_contigs, lo, hi, alpha=b"ACGT"):
    """Contigs holding copies of the queries with up to maxSubs + 1
    substitutions, either strand."""
    out = []
    for _ in range(n_contigs):
        c = bytearray(rand_dna(rng, rng.randint(lo, hi), alpha))
        for _ in range(3):
            j = rng.randrange(len(qs))
            q = qs[j]
            if len(c) < len(q):
                break
            copy = _mutate(rng, q, rng.randint(0, ks[j] + 1))
            if rng.random() < 0.5:
                copy = revcomp(copy)
            p = rng.randint(0, len(c) - len(q))
            c[p:p + len(q)] = copy
        out.append(bytes(c))
    return out


def run_indexed(ifa, qs, contigs, ks, mn=None, params=None, calls=1, **cfg):
    cfg["flags"] = cfg.get("flags", 0) | ifa.IFA_FLAG_INDEXED
    with ifa.Scanner(**cfg) as s:
        ifa.ifa_set_index_params(s.ctx, **(params or {}))
        s.load_queries(qs, ks, mn)
        k, thr = ifa.ifa_query_seeds(s.ctx, len(qs))
        parts = np.array_split(np.arange(len(contigs)), max(calls, 1)) if contigs else []
        for idx in parts:
            s.scan_chunk([contigs[i] for i in idx])
        if cfg.get("sink", 0) == ifa.IFA_SINK_COUNT_DIGEST:
            return k, thr, s.query_stats()
        return k, thr, s.collect()


def oracle_seeds(orc, qs, ks, params, strands=3):
    p = dict(params)
    kw = dict(ks=tuple(p.pop("ks", (8, 9, 10, 12, 14))), mask=p.pop("mask", 0),
              step=p.pop("step", 1), iters=p.pop("iters", 200_000), seed=p.pop("seed", 1),
              ppm=p.pop("prob_ppm", 999_000))
    assert not p
    seeds = orc.indexed_params(qs, ks, **kw)
    thr = np.array(seeds["thr"], dtype=np.uint32).reshape(-1, 2)
    for s in (0, 1):
        if not strands & (1 << s):
            thr[:, s] = 0
    return seeds, thr


@pytest.mark.parametrize("params", [
    dict(iters=3000),
    dict(iters=3000, prob_ppm=1_000_000),
    dict(iters=2000, mask=3, ks=(9, 11, 13), prob_ppm=990_000),
    dict(iters=2000, step=2, ks=(6, 8, 10)),
    # keys of 30 and 32 bits: the presence bitmap is indexed by the key's hash
    dict(iters=2000, ks=(15, 16), prob_ppm=1_000_000),
])
def test_indexed_seeds_and_hits_match_oracle(ifa, orc, params):
    rng = random.Random(3100 + len(str(params)))
    for trial in range(6):
        qs = [rand_dna(rng, rng.randint(14, 120), b"ACGT" if rng.random() < 0.8 else b"ACGTN")
              for _ in range(rng.randint(1, 12))]
        ks = [rng.randint(0, max(1, len(q) // 6)) for q in qs]
        contigs = _planted(rng, qs, ks, rng.randint(1, 6), 50, 3000,
                           rng.choice([b"ACGT", b"ACGTACGTN"]))
        strands = rng.choice([3, 3, 1, 2])
        policy = rng.choice([0, 1])
        chunk = rng.choice([4096, 1 << 16])
        say(f"indexed {params} trial {trial}: {len(qs)} queries, strands {strands}, "
            f"policy {policy}, chunk {chunk}")
        seeds, thr = oracle_seeds(orc, qs, ks, params, strands)
        k, gthr, got = run_indexed(ifa, qs, contigs, ks, params=params, strands=strands,
                                   n_policy=policy, chunk_bases=chunk,
                                   calls=rng.choice([1, 2]))
        assert list(k) == seeds["k"], trial
        assert np.array_equal(gthr, thr), trial
        want = orc.scan(qs, contigs, ks, strands=strands, policy=policy, seeds=seeds)
        assert_same(got, want, f"trial {trial}")


def test_indexed_planted_reads_are_found(ifa, orc):
    """Reads cut from the reference with up to maxSubs substitutions: every
    one is reported at its origin (the oracle agrees, and at 100 % the
    deterministic bound guarantees any copy with an error-free seed)."""
    rng = random.Random(3200)
    contigs = [rand_dna(rng, rng.randint(2000, 30000)) for _ in range(8)]
    qs, ks, origin = [], [], []
    for j in range(60):
        c = rng.randrange(len(contigs))
        L = rng.choice([30, 50, 100, 150])
        p = rng.randint(0, len(contigs[c]) - L)
        s = rng.randint(0, 4)
        q = _mutate(rng, contigs[c][p:p + L], s)
        strand = rng.randint(0, 1)
        qs.append(q if strand == 0 else revcomp(q))
        ks.append(s)
        origin.append((j, c, p, strand))
    params = dict(iters=5000, prob_ppm=1_000_000)
    say("indexed planted reads: 60 reads, 8 contigs")
    seeds, thr = oracle_seeds(orc, qs, ks, params)
    k, gthr, got = run_indexed(ifa, qs, contigs, ks, params=params, chunk_bases=1 << 16)
    want = orc.scan(qs, contigs, ks, seeds=seeds)
    assert_same(got, want, "planted")
    found = {(int(r[0]), int(r[1]), int(r[2]), int(r[3])) for r in got.tolist()}
    assert all(o in found for o in origin)


def test_indexed_overflow_and_count_digest(ifa, orc):
    rng = random.Random(3300)
    qs = [rand_dna(rng, 16, b"AC") for _ in range(4)]     # low complexity: many seeds hit
    ks = [4, 5, 6, 8]
    contigs = [rand_dna(rng, 5000, b"AC") for _ in range(3)]
    params = dict(iters=2000, ks=(8, 10))
    seeds, _ = oracle_seeds(orc, qs, ks, params)
    want, cnt, dig = orc.scan(qs, contigs, ks, seeds=seeds, stats=True)
    assert len(want) > 500
    for cap in (7, 1 << 20):
        say(f"indexed overflow: hit capacity {cap}")
        _, _, got = run_indexed(ifa, qs, contigs, ks, params=params, hit_capacity=cap,
                                chunk_bases=4096)
        assert_same(got, want, f"cap {cap}")
    say("indexed count+digest")
    _, _, (gc, gd) = run_indexed(ifa, qs, contigs, ks, params=params,
                                 sink=ifa.IFA_SINK_COUNT_DIGEST, chunk_bases=1 << 16)
    assert np.array_equal(gc, cnt) and np.array_equal(gd, dig)


def test_indexed_resident_reference(ifa, orc):
    rng = random.Random(3400)
    qs = [rand_dna(rng, rng.randint(20, 80)) for _ in range(20)]
    ks = [rng.randint(0, 6) for _ in qs]
    contigs = _planted(rng, qs, ks, 30, 1000, 40000)
    params = dict(iters=3000)
    seeds, _ = oracle_seeds(orc, qs, ks, params)
    want = orc.scan(qs, contigs, ks, seeds=seeds)
    say("indexed resident reference, eager and graph replays")
    for flags in (ifa.IFA_FLAG_INDEXED, ifa.IFA_FLAG_INDEXED | ifa.IFA_FLAG_GRAPHS):
        with ifa.Scanner(chunk_bases=1 << 18, flags=flags) as s:
            ifa.ifa_set_index_params(s.ctx, **params)
            s.ref_load(contigs)
            for rep in range(3):
                s.load_queries(qs, ks)
                s.scan_resident()
                assert_same(s.collect(), want, f"flags {flags} rep {rep}")


def test_indexed_errors(ifa):
    say("indexed mode errors")
    with ifa.Scanner(chunk_bases=4096) as s:
        with pytest.raises(ifa.IfaError):           # not an indexed context
            ifa.ifa_set_index_params(s.ctx, iters=10)
    with ifa.Scanner(chunk_bases=4096, flags=ifa.IFA_FLAG_INDEXED) as s:
        for bad in (dict(ks=(17,)), dict(ks=()), dict(step=0), dict(prob_ppm=1_000_001),
                    dict(mask=8, ks=(8,)), dict(iters=0)):
            with pytest.raises(ifa.IfaError):
                ifa.ifa_set_index_params(s.ctx, **bad)
        ifa.ifa_set_index_params(s.ctx, mask=4, ks=(9,), iters=100)
        with pytest.raises(ifa.IfaError):           # query not longer than the mask
            s.load_queries([b"ACGT"], [0])


def test_auto_mode_follows_the_query_count(ifa, orc):
    """IFA_FLAG_AUTO_MODE: a query set below auto_queries runs by brute force
    (the brute-force oracle's hits), one at or above it in indexed mode (the
    indexed oracle's hits); the same context switches between them."""
    rng = random.Random(3500)
    qs = [rand_dna(rng, rng.randint(20, 60)) for _ in range(12)]
    ks = [rng.randint(0, 5) for _ in qs]
    contigs = _planted(rng, qs, ks, 20, 500, 20000)
    params = dict(iters=2000, auto_queries=8)
    with ifa.Scanner(chunk_bases=1 << 18, flags=ifa.IFA_FLAG_AUTO_MODE) as s:
        ifa.ifa_set_index_params(s.ctx, **params)
        s.ref_load(contigs)
        for n in (3, 12, 7, 8):
            say(f"auto mode: {n} queries")
            s.load_queries(qs[:n], ks[:n])
            s.scan_resident()
            got = s.collect()
            p = dict(params)
            p.pop("auto_queries")
            if n >= 8:
                assert ifa.ifa_query_mode(s.ctx) == 1
                seeds, _ = oracle_seeds(orc, qs[:n], ks[:n], p)
                want = orc.scan(qs[:n], contigs, ks[:n], seeds=seeds)
            else:
                assert ifa.ifa_query_mode(s.ctx) == 0
                want = orc.scan(qs[:n], contigs, ks[:n])
            assert_same(got, want, f"auto {n}")


def test_indexed_many_queries(ifa, orc):
    """2,000 reads cut from the reference with up to 4 substitutions: the seed
    tables hold a few hundred thousand entries, so the host builds them in
    many slices and every one of the 256 top-bit partitions. Seed lengths,
    thresholds and hits match the oracle's."""
    rng = random.Random(3600)
    contigs = [rand_dna(rng, 60000) for _ in range(2)]
    qs = []
    for _ in range(2000):
        c = rng.randrange(2)
        L = rng.choice([60, 100])
        p = rng.randint(0, 60000 - L)
        q = bytearray(contigs[c][p:p + L])
        for i in rng.sample(range(L), rng.randint(0, 4)):
            q[i] = rng.choice(b"ACGT")
        qs.append(bytes(q) if rng.random() < 0.5 else revcomp(bytes(q)))
    ks = [rng.randint(0, 4) for _ in qs]
    params = dict(iters=2000)
    seeds, thr = oracle_seeds(orc, qs, ks, params)
    want = orc.scan(qs, contigs, ks, seeds=seeds)
    assert len(want) >= 1000
    say("indexed mode, 2,000 queries")
    k, gthr, got = run_indexed(ifa, qs, contigs, ks, params=params, chunk_bases=1 << 16)
    assert list(k) == seeds["k"]
    assert np.array_equal(gthr, thr)
    assert_same(got, want, "2,000 queries")
