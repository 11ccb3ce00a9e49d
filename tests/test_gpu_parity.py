"""Parity of the HIP scan (through the C ABI) with the oracle.

Every comparison is element by element on all six record fields (query,
contig, pos, strand, n_ref, mismatches) in reference order; the method is
integer-only, so the bar is bit-exact. Inputs are seeded; each test prints the
case it is about to run before touching the GPU.
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


def gpu_scan(ifa, queries, contigs, ks, mn=None, *, calls=1, **cfg):
    with ifa.Scanner(**cfg) as s:
        s.load_queries(queries, ks, mn)
        if calls <= 1:
            s.scan_chunk(contigs)
        else:
            parts = np.array_split(np.arange(len(contigs)), calls)
            for idx in parts:
                s.scan_chunk([contigs[i] for i in idx])
        return s.collect()


def assert_same(a, b, ctx=""):
    if not np.array_equal(a, b):
        sa = {tuple(r) for r in a.tolist()}
        sb = {tuple(r) for r in b.tolist()}
        raise AssertionError(f"{ctx}: gpu {len(a)} oracle {len(b)}; only gpu "
                             f"{sorted(sa - sb)[:5]} only oracle {sorted(sb - sa)[:5]}")


def test_c1_tiny_bit_exact(ifa, orc):
    import synth
    w = synth.c1_tiny()
    say("c1_tiny: 1 query L32 vs 10 x 100 kbp, k=3")
    want = orc.scan(w.queries, w.ref, w.max_subs)
    got = gpu_scan(ifa, w.queries, w.ref, w.max_subs)
    assert_same(got, want, "c1")
    assert len(got) == 20
    planted = {(p.query, p.contig, p.pos, p.strand, 0, p.subs) for p in w.plants}
    assert {tuple(r) for r in got.tolist()} == planted


@pytest.mark.parametrize("policy", [0, 1])
def test_random_small_cases(ifa, orc, policy):
    rng = random.Random(1000 + policy)
    for trial in range(60):
        nc = rng.randint(0, 6)
        contigs = []
        for _ in range(nc):
            n = rng.choice([0, 1, 5, 31, 32, 33, 63, 64, 65, 100, 257, 1000, 4000])
            alpha = rng.choice([b"ACGT", b"ACGT", b"ACGTN", b"acgtNNRY"])
            contigs.append(rand_dna(rng, n, alpha))
        nq = rng.randint(1, 6)
        qs = [rand_dna(rng, rng.choice([1, 2, 7, 16, 31, 32, 33, 40, 63, 64, 65, 100]),
                       b"ACGT" if rng.random() < 0.85 else b"ACGTN") for _ in range(nq)]
        ks = [rng.randint(0, len(q) + 1) if rng.random() < 0.5 else rng.randint(0, 3) for q in qs]
        mn = None if rng.random() < 0.5 else [rng.randint(0, len(q)) for q in qs]
        strands = rng.choice([1, 2, 3])
        chunk = rng.choice([4096, 4096 + 32 * 7, 1 << 16])
        say(f"random trial {trial} policy {policy} nq {nq} nc {nc} chunk {chunk}")
        want = orc.scan(qs, contigs, ks, mn, strands=strands, policy=policy)
        got = gpu_scan(ifa, qs, contigs, ks, mn, strands=strands, n_policy=policy,
                       chunk_bases=chunk, calls=rng.choice([1, 2, 3]))
        assert_same(got, want, f"trial {trial}")


def test_queries_of_every_length_and_threshold(ifa, orc):
    rng = random.Random(77)
    contigs = [rand_dna(rng, 3000, b"ACGTN") for _ in range(3)]
    for L in (1, 2, 3, 8, 15, 31, 32, 33, 47, 64, 95, 96, 97, 128, 150, 200, 254, 255):
        # plant a few near copies so high-threshold and low-threshold hits exist
        q = rand_dna(rng, L)
        cs = []
        for c in contigs:
            c = bytearray(c)
            for _ in range(3):
                p = rng.randint(0, len(c) - L)
                src = q if rng.random() < 0.5 else q.translate(COMP)[::-1]
                c[p:p + L] = src
            cs.append(bytes(c))
        ks = [0, L // 8, L // 4, L // 2, L]
        say(f"length {L}")
        want = orc.scan([q] * len(ks), cs, ks)
        got = gpu_scan(ifa, [q] * len(ks), cs, ks, chunk_bases=8192)
        assert_same(got, want, f"L={L}")


def test_chunk_size_and_call_split_invariance(ifa, orc):
    import synth
    spec = synth.c2_spec(seed=21, total=3_000_000)
    spec.n_param = 2e-3
    spec.median = 20_000
    ref = synth.gen_reference(spec)
    qs = synth.gen_queries(21, 6, 20, 60)
    ks = [6, 8, 10, 12, 14, 16]
    say("chunk invariance: 3 Mbp, 6 queries")
    want = orc.scan(qs, ref, ks)
    contigs = [ref.contig(i) for i in range(ref.n_contigs)]
    for chunk, calls in ((4096, 1), (4096 + 32, 5), (100_000, 3), (1 << 20, 2), (1 << 30, 1)):
        say(f"  chunk {chunk} calls {calls}")
        got = gpu_scan(ifa, qs, contigs, ks, chunk_bases=chunk, calls=calls)
        assert_same(got, want, f"chunk {chunk}")


def test_contig_longer_than_chunk(ifa, orc):
    rng = random.Random(5)
    q = rand_dna(rng, 40)
    big = bytearray(rand_dna(rng, 50_000, b"ACGTN"))
    for p in range(0, 50_000 - 40, 997):       # copies straddling every chunk boundary
        big[p:p + 40] = q
    contigs = [rand_dna(rng, 100), bytes(big), rand_dna(rng, 10)]
    say("contig longer than chunk")
    want = orc.scan([q], contigs, [2])
    got = gpu_scan(ifa, [q], contigs, [2], chunk_bases=4096)
    assert_same(got, want, "long contig")
    assert len(got) >= 50


def test_overflow_rescan_gives_same_result(ifa, orc):
    rng = random.Random(8)
    contigs = [rand_dna(rng, 20_000) for _ in range(3)]
    qs = [rand_dna(rng, 10), rand_dna(rng, 12)]
    ks = [5, 6]                 # thousands of hits
    say("overflow: hit capacity 7")
    want = orc.scan(qs, contigs, ks)
    assert len(want) > 1000
    for cap in (7, 100, 1 << 20):
        got = gpu_scan(ifa, qs, contigs, ks, hit_capacity=cap, chunk_bases=16384)
        assert_same(got, want, f"cap {cap}")


@pytest.mark.parametrize("policy", [0, 1])
def test_count_digest_sink(ifa, orc, policy):
    import synth
    spec = synth.c2_spec(seed=33, total=2_000_000)
    spec.n_param = 1e-3
    ref = synth.gen_reference(spec)
    qs = synth.gen_queries(33, 40, 18, 50)
    rng = np.random.default_rng(33)
    ks = [int(x) for x in rng.integers(0, 17, size=len(qs))]
    say(f"count+digest policy {policy}")
    _, cnt, dig = orc.scan(qs, ref, ks, policy=policy, stats=True, records=False)
    with ifa.Scanner(sink=ifa.IFA_SINK_COUNT_DIGEST, n_policy=policy, chunk_bases=1 << 18) as s:
        s.load_queries(qs, ks)
        s.scan_chunk(ref)
        gc, gd = s.query_stats()
    assert np.array_equal(gc, cnt)
    assert np.array_equal(gd, dig)
    assert int(cnt.sum()) > 10_000


def test_resident_reference_matches_streaming(ifa, orc):
    import synth
    spec = synth.c2_spec(seed=44, total=5_000_000)
    ref = synth.gen_reference(spec)
    rng = random.Random(44)
    say("resident reference, two query sets")
    with ifa.Scanner(chunk_bases=1 << 21) as s:
        first = s.ref_load(ref)
        assert first == 0
        bases, chunks = ifa.ifa_ref_info(s.ctx)
        assert bases == ref.total and chunks == 3
        for round_ in range(2):
            qs = [rand_dna(rng, rng.randint(18, 60)) for _ in range(5)]
            ks = [rng.randint(2, 12) for _ in qs]
            s.load_queries(qs, ks)
            s.scan_resident()
            got = s.collect()
            want = orc.scan(qs, ref, ks)
            assert_same(got, want, f"resident round {round_}")


def test_error_paths(ifa):
    say("error paths")
    with ifa.Scanner(chunk_bases=4096) as s:
        with pytest.raises(ifa.IfaError) as e:
            s.load_queries([b""], [0])
        assert e.value.status == 5
        with pytest.raises(ifa.IfaError) as e:
            s.load_queries([b"A" * 257], [0])
        assert e.value.status == 5
        with pytest.raises(ifa.IfaError) as e:
            s.load_queries([b"A" * 256], [0])    # n_ref would not fit its byte
        assert e.value.status == 5
        with pytest.raises(ifa.IfaError) as e:
            s.load_queries([b"ACGT"], [-1])
        assert e.value.status == 1
        with pytest.raises(ifa.IfaError) as e:
            s.scan_chunk([b"ACGT"])              # no queries yet
        assert e.value.status == 4
        s.load_queries([b"ACGT"], [0])
        s.scan_chunk([b"TTACGTT"])
        with pytest.raises(ifa.IfaError) as e:
            s.load_queries([b"ACGT"], [0])       # hits pending
        assert e.value.status == 4
        got = s.collect()
        assert {tuple(r) for r in got.tolist()} == {(0, 0, 2, 0, 0, 0), (0, 0, 2, 1, 0, 0)}
        s.load_queries([b"ACGT"], [0])           # allowed again once drained
        assert s.scan_chunk([b"", b"ACGTACGT"]) == 1     # ordinals continue
        got = s.collect()
        assert {tuple(r) for r in got.tolist()} == {(0, 2, p, st, 0, 0) for p in (0, 4)
                                                    for st in (0, 1)}


def test_collect_in_small_batches(ifa, orc):
    rng = random.Random(9)
    contigs = [rand_dna(rng, 5000) for _ in range(2)]
    qs = [rand_dna(rng, 8)]
    want = orc.scan(qs, contigs, [3])
    say("two-call drain")
    with ifa.Scanner(chunk_bases=4096) as s:
        s.load_queries(qs, [3])
        s.scan_chunk(contigs)
        parts = []
        while True:
            h, rem = ifa.ifa_collect_hits(s.ctx, 37)
            parts.append(h)
            if rem == 0:
                break
        got = np.concatenate(parts)
    assert_same(got, want, "batched drain")


def test_c2_scaled_full_parity(ifa, orc):
    """The paper-scale generator at 200 Mbp: every query and threshold of the
    configuration, full oracle comparison."""
    import synth
    say("c2 scaled: 200 Mbp, 10 queries, k in 0 4 8")
    w = synth.c2_paper_scale(total=200_000_000, plants_per_query=4)
    for k in (0, 4, 8):
        ks = [k] * len(w.queries)
        want = orc.scan(w.queries, w.ref, ks)
        with ifa.Scanner() as s:
            s.load_queries(w.queries, ks)
            s.scan_chunk(w.ref)
            got = s.collect()
        assert_same(got, want, f"c2 k={k}")
        found = {(int(r[0]), int(r[1]), int(r[2]), int(r[3])) for r in got.tolist()}
        for p in w.plants:
            if p.subs <= k:
                assert (p.query, p.contig, p.pos, p.strand) in found


def test_default_variant_is_the_three_class_matrix_filter(ifa):
    with ifa.Scanner() as s:
        v = ifa.ifa_get_variant(s.ctx)
        assert ifa.ifa_variant_info(v)["encoding"] == 2


def test_every_kernel_variant_is_bit_exact(ifa, orc):
    """The autotuner may pick any variant, so each must give the oracle's hits."""
    import synth
    spec = synth.c2_spec(seed=55, total=1_500_000)
    spec.n_param = 3e-3
    spec.median = 50_000
    ref = synth.gen_reference(spec)
    rng = random.Random(55)
    qs = [rand_dna(rng, rng.choice([5, 18, 31, 32, 33, 50, 64, 100]),
                   b"ACGT" if rng.random() < 0.9 else b"ACGTN") for _ in range(13)]
    ks = [rng.randint(0, min(len(q), 12)) for q in qs]
    want = orc.scan(qs, ref, ks)
    _, cnt, dig = orc.scan(qs, ref, ks, stats=True, records=False)
    for v in range(ifa.ifa_variant_count()):
        say(f"variant {v} {ifa.ifa_variant_info(v)}")
        with ifa.Scanner(chunk_bases=1 << 19) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            s.scan_chunk(ref)
            assert_same(s.collect(), want, f"variant {v}")
        with ifa.Scanner(chunk_bases=1 << 19, sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            s.scan_chunk(ref)
            gc, gd = s.query_stats()
            assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"variant {v} stats"


def test_autotune_chooses_a_variant_and_caches_it(ifa, orc, tmp_path):
    rng = random.Random(66)
    qs = [rand_dna(rng, 32) for _ in range(8)]
    ks = [3] * 8
    cache = str(tmp_path / "tune.txt")
    say("autotune")
    with ifa.Scanner(chunk_bases=1 << 22) as s:
        s.load_queries(qs, ks)
        v, ms = ifa.ifa_autotune(s.ctx, 1 << 22, 3, cache)
        assert 0 <= v < ifa.ifa_variant_count()
        assert ms[v] > 0 and ms[v] == ms[ms > 0].min()
        assert ifa.ifa_get_variant(s.ctx) == v
        ifa.ifa_set_variant(s.ctx, 0)
        v2, ms2 = ifa.ifa_autotune(s.ctx, 1 << 22, 3, cache)      # cache hit
        assert v2 == v and (ms2 == -1).all()
        # tuning leaves no hits behind; a scan after it is exact
        c = rand_dna(rng, 20000)
        s.scan_chunk([c])
        assert_same(s.collect(), orc.scan(qs, [c], ks), "after autotune")


@pytest.mark.parametrize("sink", [0, 1])
def test_dense_and_sparse_strands_with_work_list_overflow(ifa, orc, sink):
    """A query set mixing filtered (sparse) and hit-dense strands, lengths 18-150
    and thresholds up to L/2; a work list of 4 items forces the grow-and-rerun
    path of the filtered part. Records and count+digest must both match."""
    import synth
    spec = synth.c2_spec(seed=77, total=600_000)
    spec.n_param = 2e-3
    spec.median = 40_000
    ref = synth.gen_reference(spec)
    rng = random.Random(77)
    qs = [rand_dna(rng, rng.choice([18, 20, 24, 31, 32, 33, 40, 50, 64, 100, 150]))
          for _ in range(24)]
    ks = [rng.randint(0, len(q) // 2) for q in qs]
    say(f"dense+sparse mix, sink {sink}")
    want, cnt, dig = orc.scan(qs, ref, ks, stats=True)
    for wcap in (4, 0):
        with ifa.Scanner(chunk_bases=1 << 18, work_capacity=wcap, sink=sink,
                         hit_capacity=1 << 14) as s:
            s.load_queries(qs, ks)
            s.scan_chunk(ref)
            if sink == 0:
                assert_same(s.collect(), want, f"records wcap {wcap}")
            else:
                gc, gd = s.query_stats()
                assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"stats wcap {wcap}"
            st = s.stats()
            if wcap == 4:
                assert st["rescans"] > 0
    assert len(want) > 1000


@pytest.mark.parametrize("n_two,n_one", [(40, 0), (16, 20), (17, 20)])
def test_two_word_batches_run_their_own_launch(ifa, orc, n_two, n_one):
    """Strands filtered on a 64-base prefix (L 64, maxSubs 16) sort ahead of
    the one-word ones (L 30, maxSubs 2), and the batches of 32 strands holding
    them run the two-word filter while the rest run the one-word filter:
    every batch two-word; two-word strands filling exactly one batch; and one
    query more, so that a batch mixes both kinds."""
    import synth
    spec = synth.c2_spec(seed=95, total=800_000)
    spec.n_param = 1e-3
    ref = synth.gen_reference(spec)
    rng = random.Random(95 + n_two + n_one)
    qs = [rand_dna(rng, 64) for _ in range(n_two)] + [rand_dna(rng, 30) for _ in range(n_one)]
    ks = [16] * n_two + [2] * n_one
    buf = bytearray(ref.buf.tobytes())
    for qi, q in enumerate(qs):          # near copies, so that both kinds have hits
        c = rng.randrange(ref.n_contigs)
        n = int(ref.lens[c])
        p = int(ref.offs[c]) + rng.randint(0, n - len(q))
        src = bytearray(q if qi % 2 else q.translate(COMP)[::-1])
        for j in rng.sample(range(len(q)), ks[qi]):
            src[j] = rng.choice(b"ACGT")
        buf[p:p + len(q)] = src
    ref = synth.Reference(np.frombuffer(bytes(buf), dtype=np.uint8).copy(), ref.offs, ref.lens)
    want = orc.scan(qs, ref, ks)
    assert len(want) >= len(qs)
    for v in range(ifa.ifa_variant_count()):
        if ifa.ifa_variant_info(v)["encoding"] not in (2, 3):
            continue
        say(f"two-word batches: {n_two} two-word, {n_one} one-word queries, variant {v}")
        with ifa.Scanner(chunk_bases=1 << 18) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            strands, filtered = ifa.ifa_query_partition(s.ctx)
            assert (strands, filtered) == (2 * len(qs), 2 * len(qs))
            s.scan_chunk(ref)
            assert_same(s.collect(), want, f"variant {v}")


def test_dense_strands_where_every_window_hits(ifa, orc):
    """maxSubs >= L: every window of every plain lane is a hit, so the dense
    kernel's per-wave hit list is full (64 lanes x W windows) for every
    strand; N runs and contig ends send some lanes to the cold kernel.
    Count+digest for one variant of each lane width."""
    import synth
    spec = synth.c2_spec(seed=91, total=1_200_000)
    spec.n_param = 2e-3
    spec.median = 60_000
    ref = synth.gen_reference(spec)
    rng = random.Random(91)
    qs = [rand_dna(rng, L) for L in (6, 12, 18, 25, 32, 33, 47)]
    ks = [len(q) + rng.randint(0, 3) for q in qs]
    _, cnt, dig = orc.scan(qs, ref, ks, stats=True, records=False)
    widths = {}
    for v in range(ifa.ifa_variant_count()):
        widths.setdefault(ifa.ifa_variant_info(v)["windows_per_lane"], v)
    assert len(widths) >= 2
    for w, v in sorted(widths.items()):
        say(f"every window hits: variant {v} (W {w})")
        with ifa.Scanner(chunk_bases=1 << 18, sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            strands, filtered = ifa.ifa_query_partition(s.ctx)
            assert filtered == 0
            s.scan_chunk(ref)
            gc, gd = s.query_stats()
        assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"variant {v}"
    assert int(cnt.sum()) > 10_000_000


def matrix_variants(ifa):
    return [v for v in range(ifa.ifa_variant_count()) if ifa.ifa_variant_info(v)["encoding"] >= 1]


@pytest.mark.parametrize("strands,policy", [(1, 0), (3, 1)])
def test_matrix_core_filter_cases(ifa, orc, strands, policy):
    """The fp4 matrix-core filter on the cases its tiling has to get right:
    strand counts that are odd (a half-empty column tile) and span several
    batches of 32, lengths below, at and above 32 with query Ns, thresholds
    0-12, reference N runs and several chunks. Small hit buffers and work
    lists force the re-scan and re-run paths through the same kernel."""
    import synth
    spec = synth.c2_spec(seed=91, total=900_000)
    spec.n_param = 3e-3
    spec.median = 60_000
    ref = synth.gen_reference(spec)
    rng = random.Random(91 + strands)
    qs = [rand_dna(rng, rng.choice([5, 12, 18, 24, 31, 32, 33, 36, 47, 64, 100]),
                   b"ACGT" if rng.random() < 0.85 else b"ACGTN") for _ in range(45)]
    ks = [rng.randint(0, min(len(q), 12)) for q in qs]
    want = orc.scan(qs, ref, ks, strands=strands, policy=policy)
    _, cnt, dig = orc.scan(qs, ref, ks, strands=strands, policy=policy, stats=True, records=False)
    vs = matrix_variants(ifa)
    assert vs, "no matrix-core variant"
    for v in vs:
        for hcap, wcap in ((1 << 20, 0), (1 << 9, 8)):
            say(f"matrix variant {v} strands {strands} policy {policy} hcap {hcap} wcap {wcap}")
            with ifa.Scanner(chunk_bases=1 << 18, strands=strands, n_policy=policy,
                             hit_capacity=hcap, work_capacity=wcap) as s:
                ifa.ifa_set_variant(s.ctx, v)
                s.load_queries(qs, ks)
                s.scan_chunk(ref)
                assert_same(s.collect(), want, f"variant {v} hcap {hcap} wcap {wcap}")
        with ifa.Scanner(chunk_bases=1 << 18, strands=strands, n_policy=policy,
                         sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            s.scan_chunk(ref)
            gc, gd = s.query_stats()
            assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"variant {v} stats"
    assert len(want) > 200


def test_matrix_core_filter_emits_what_the_valu_filter_emits(ifa):
    """The VALU and four-class filters compute the same count and test N per
    plane word, so on the same chunk they list the same work items (same
    waves, batches and pending strands) and skip the same N waves: compared
    through the library's counters. The three-class filter takes N from
    32-word block flags, which may also send waves without an N to the exact
    path: its variants agree with each other and evaluate at most the
    windows of the others, nearly all of them."""
    import synth
    spec = synth.c2_spec(seed=5, total=3_000_000)
    spec.n_param = 1e-3
    ref = synth.gen_reference(spec)
    rng = random.Random(5)
    qs = [rand_dna(rng, rng.choice([20, 28, 32, 40])) for _ in range(40)]
    ks = [rng.randint(2, 7) for _ in qs]
    seen = {}
    for v in range(ifa.ifa_variant_count()):
        info = ifa.ifa_variant_info(v)
        if info["windows_per_lane"] != 16:
            continue
        say(f"work items of variant {v} {info}")
        with ifa.Scanner(chunk_bases=1 << 20) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            s.scan_chunk(ref)
            s.collect()
            st = s.stats()
            seen[v] = (st["work_items"], st["filter_windows"], info["encoding"])
    word = {x[:2] for x in seen.values() if x[2] < 2}
    block = {x[:2] for x in seen.values() if x[2] >= 2}
    assert len(word) == 1 and len(block) == 1, seen
    (_, w_word), (_, w_block) = word.pop(), block.pop()
    assert 0.98 * w_word <= w_block <= w_word, seen


@pytest.mark.parametrize("sink", [0, 1])
def test_resident_graph_replays_match_eager(ifa, orc, sink):
    """Resident passes replayed from captured graphs give the eager results on
    every replay, also after the query data changes under the same launch
    arguments; eager scans by another context run between the replays."""
    import synth
    spec = synth.c2_spec(seed=66, total=3_000_000)
    spec.n_param = 2e-3
    spec.median = 100_000
    ref = synth.gen_reference(spec)
    rng = random.Random(66)
    lens = [rng.choice([24, 31, 32, 36, 40]) for _ in range(12)]
    qa = [rand_dna(rng, n) for n in lens]
    qb = [rand_dna(rng, n) for n in lens]          # same shapes, other bases
    ks = [rng.randint(0, 6) for _ in lens]
    want = {}
    for name, qs in (("a", qa), ("b", qb)):
        if sink == 0:
            want[name] = orc.scan(qs, ref, ks)
        else:
            _, cnt, dig = orc.scan(qs, ref, ks, stats=True, records=False)
            want[name] = (cnt, dig)
    cfg = dict(chunk_bases=1 << 20, sink=sink)
    with ifa.Scanner(flags=ifa.IFA_FLAG_GRAPHS, **cfg) as g, ifa.Scanner(flags=0, **cfg) as e:
        g.ref_load(ref)
        e.ref_load(ref)
        for rep, name in enumerate(["a", "a", "a", "b", "a", "b"]):
            qs = qa if name == "a" else qb
            say(f"graph replay {rep} queries {name} sink {sink}")
            for s in (g, e):
                s.load_queries(qs, ks)
                s.scan_resident()
                if sink == 0:
                    assert_same(s.collect(), want[name], f"rep {rep} {name}")
                else:
                    gc, gd = s.query_stats()
                    assert np.array_equal(gc, want[name][0]) and np.array_equal(gd, want[name][1])
        st = g.stats()
        assert st["graph_launches"] > 0
        assert e.stats()["graph_launches"] == 0


@pytest.mark.parametrize("sink", [0, 1])
def test_forked_pass_graphs_with_dense_strands(ifa, orc, sink):
    """Passes holding both filtered and dense strands run the dense kernels on
    a second stream beside the filter; their captured graphs fork and join.
    Streamed chunks replayed with the kernel nodes pointed at each new chunk,
    for two query sets in turn, give the oracle's results, for the default
    variant, a VALU variant and the variant that counts dense strands on the
    matrix cores."""
    import synth
    spec = synth.c2_spec(seed=88, total=2_200_000)
    spec.n_param = 2e-3
    spec.median = 80_000
    ref = synth.gen_reference(spec)
    contigs = [ref.contig(i) for i in range(ref.n_contigs)]
    rng = random.Random(88)
    shape = [(18, 10), (20, 9), (22, 8), (24, 12), (30, 14), (31, 3), (36, 5), (40, 7), (64, 9)]
    sets = []
    for _ in range(2):
        qs = [rand_dna(rng, L) for L, _ in shape for _ in range(2)]
        ks = [k for _, k in shape for _ in range(2)]
        sets.append((qs, ks))
    order = [0, 1, 0]
    want = []
    for rep, i in enumerate(order):
        # each scan of a context numbers its contigs after the earlier ones
        first = rep * len(contigs)
        if sink == 0:
            want.append(orc.scan(sets[i][0], contigs, sets[i][1], first_ordinal=first))
        else:
            _, cnt, dig = orc.scan(sets[i][0], contigs, sets[i][1], stats=True, records=False,
                                   first_ordinal=first)
            want.append((cnt, dig))
    info = [ifa.ifa_variant_info(v) for v in range(ifa.ifa_variant_count())]
    variants = [None, next(v for v, x in enumerate(info) if x["encoding"] == 0),
                next(v for v, x in enumerate(info) if x["encoding"] == 3)]
    for v in variants:
        with ifa.Scanner(chunk_bases=1 << 17, sink=sink, flags=ifa.IFA_FLAG_GRAPHS) as s:
            if v is None:
                v = ifa.ifa_get_variant(s.ctx)
            ifa.ifa_set_variant(s.ctx, v)
            for rep, i in enumerate(order):
                say(f"forked pass graphs: variant {v} sink {sink} rep {rep} set {i}")
                s.load_queries(*sets[i])
                strands, filtered = ifa.ifa_query_partition(s.ctx)
                assert 0 < filtered < strands
                s.scan_chunk(contigs)
                if sink == 0:
                    assert_same(s.collect(), want[rep], f"variant {v} rep {rep}")
                else:
                    gc, gd = s.query_stats()
                    assert np.array_equal(gc, want[rep][0]) and \
                        np.array_equal(gd, want[rep][1]), f"variant {v} rep {rep}"
            st = s.stats()
            assert st["graph_launches"] > 0 and st["graph_updates"] > 0, (v, st)


def test_overlap_switched_off_and_on(ifa, orc):
    """ifa_set_overlap: passes with both filtered and dense strands give the
    oracle's hits with the dense kernels beside the filter and after it, from
    captured graphs (captured again when the arrangement changes) and
    eagerly."""
    import synth
    spec = synth.c2_spec(seed=99, total=1_500_000)
    spec.n_param = 2e-3
    spec.median = 70_000
    ref = synth.gen_reference(spec)
    rng = random.Random(99)
    shape = [(18, 10), (21, 9), (26, 12), (33, 4), (40, 6), (64, 8)]
    qs = [rand_dna(rng, L) for L, _ in shape for _ in range(3)]
    ks = [k for _, k in shape for _ in range(3)]
    want = orc.scan(qs, ref, ks)
    with ifa.Scanner(chunk_bases=1 << 19, flags=ifa.IFA_FLAG_GRAPHS) as s:
        s.ref_load(ref)
        s.load_queries(qs, ks)
        strands, filtered = ifa.ifa_query_partition(s.ctx)
        assert 0 < filtered < strands
        for graphs in (True, False):
            ifa.ifa_set_graphs(s.ctx, graphs)
            for overlap in (True, False, True):
                ifa.ifa_set_overlap(s.ctx, overlap)
                for i in range(3):
                    say(f"overlap {overlap} graphs {graphs} pass {i}")
                    s.scan_resident()
                    assert_same(s.collect(), want, f"overlap {overlap} graphs {graphs} pass {i}")
            if graphs:
                assert s.stats()["graph_launches"] > 0


@pytest.mark.parametrize("sink", [0, 1])
def test_streamed_graph_replays_match_eager(ifa, orc, sink):
    """Streamed chunks (two stream slots, two hit buffers) replayed from
    captured pass graphs whose kernel nodes are pointed at each new chunk
    (other lengths, carried prefixes, piece tables) give the eager results,
    for two query sets in turn (other tables, counts and launch grids), with
    a hit-buffer overflow in records mode."""
    import synth
    spec = synth.c2_spec(seed=67, total=2_500_000)
    spec.n_param = 2e-3
    spec.median = 60_000
    ref = synth.gen_reference(spec)
    contigs = [ref.contig(i) for i in range(ref.n_contigs)]
    rng = random.Random(67)
    sets = []
    for n in (10, 23):
        lens = [rng.choice([18, 24, 31, 32, 36, 40, 70]) for _ in range(n)]
        sets.append(([rand_dna(rng, x) for x in lens], [rng.randint(0, 8) for _ in lens]))
    cfg = dict(chunk_bases=1 << 17, sink=sink, hit_capacity=5000 if sink == 0 else 0)
    for rep, (qs, ks) in enumerate(sets + sets):
        say(f"streamed graph replay {rep} sink {sink}")
        # the third scan of the context numbers its contigs after the first two
        first = 2 * len(contigs)
        if sink == 0:
            want = orc.scan(qs, contigs, ks, first_ordinal=first)
        else:
            _, cnt, dig = orc.scan(qs, contigs, ks, stats=True, records=False,
                                   first_ordinal=first)
        with ifa.Scanner(flags=ifa.IFA_FLAG_GRAPHS, **cfg) as g:
            for qs_, ks_ in ((qs, ks), sets[(rep + 1) % 2], (qs, ks)):
                g.load_queries(qs_, ks_)
                g.scan_chunk(contigs)
                if sink == 0:
                    got = g.collect()
                else:
                    gc, gd = g.query_stats()
            st = g.stats()
        if sink == 0:
            assert_same(got, want, f"rep {rep}")
        else:
            assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"rep {rep}"
        assert st["graph_launches"] > 0 and st["graph_updates"] > 0, st


@pytest.mark.parametrize("sink", [0, 1])
def test_two_word_filter_prefix(ifa, orc, sink):
    """Long queries with thresholds the 32-base prefix cannot filter (the
    three-class matrix filter then reads 64 bases; column tiles mixing one-
    and two-word strands share a launch) match the oracle under every
    variant, and those strands leave the dense path."""
    import synth
    spec = synth.c2_spec(seed=123, total=1_200_000)
    spec.n_param = 3e-3
    spec.median = 80_000
    ref = synth.gen_reference(spec)
    rng = random.Random(123)
    qs, ks = [], []
    for _ in range(30):
        L = rng.choice([33, 40, 47, 56, 64, 90, 150])
        qs.append(rand_dna(rng, L, b"ACGT" if rng.random() < 0.85 else b"ACGTN"))
        ks.append(rng.randint(min(L // 4, 20), min(L // 3 + 2, 24)))
    for _ in range(10):   # strands a 32-base prefix filters on its own
        qs.append(rand_dna(rng, rng.choice([28, 32, 36])))
        ks.append(rng.randint(0, 6))
    # the partition rule: the shortest prefix of one or two 32-base words
    # whose filter passes a window in under 1/32 of the 1024-window waves
    from scipy.stats import binom

    def words(L, k):
        for w in (1, 2):
            lf = min(L, 32 * w)
            if min(k, L) < lf and binom.cdf(min(k, L), lf, 0.75) * 1024 < 1 / 32:
                return w
            if lf == L:
                break
        return 0
    fws = [words(len(q), k) for q, k in zip(qs, ks)]
    assert fws.count(2) >= 10
    # plant near copies so that hits exist for the long queries too
    buf = bytearray(ref.buf.tobytes())
    for qi, q in enumerate(qs[:30]):
        for _ in range(2):
            c = rng.randrange(ref.n_contigs)
            n = int(ref.lens[c])
            if n < len(q) + 10:
                continue
            p = int(ref.offs[c]) + rng.randint(0, n - len(q))
            src = bytearray(q if rng.random() < 0.5 else q.translate(COMP)[::-1])
            for j in rng.sample(range(len(q)), min(len(q), ks[qi])):
                src[j] = rng.choice(b"ACGT")
            buf[p:p + len(q)] = src
    ref = synth.Reference(np.frombuffer(bytes(buf), dtype=np.uint8).copy(), ref.offs, ref.lens)
    if sink == 0:
        want = orc.scan(qs, ref, ks)
        assert len(want) > 30
    else:
        _, cnt, dig = orc.scan(qs, ref, ks, stats=True, records=False)
    for v in range(ifa.ifa_variant_count()):
        info = ifa.ifa_variant_info(v)
        if info["encoding"] == 0 and info["workgroup"] != 256:
            continue   # VALU shapes: one is enough here (they filter on 32 bases)
        say(f"two-word prefix, variant {v} {info} sink {sink}")
        with ifa.Scanner(chunk_bases=1 << 19, sink=sink) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            strands, filtered = ifa.ifa_query_partition(s.ctx)
            assert (strands, filtered) == (2 * len(qs), 2 * sum(1 for w in fws if w))
            s.scan_chunk(ref)
            if sink == 0:
                assert_same(s.collect(), want, f"variant {v}")
            else:
                gc, gd = s.query_stats()
                assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"variant {v}"


@pytest.mark.parametrize("policy", [0, 1])
def test_n_in_the_last_word_a_two_word_window_reads(ifa, orc, policy):
    """A window filtered on two prefix words (L = 64) that starts in the last
    8 starts of a 1024-window filter wave reads plane word w0 + 33 of the wave.
    A reference N there must be seen (an N byte's own bits read as G), so each
    copy below, with exactly k substitutions and one N at a strand base other
    than G in that word, is a hit under the default N rule. Every three-class
    matrix variant is run."""
    rng = random.Random(9033)
    L = 64
    q = rand_dna(rng, L)
    rc = q.translate(COMP)[::-1]
    contig = bytearray(rand_dna(rng, 16 * 1024 + 200))
    for i, s in enumerate(range(1016, 1024)):
        start = 2048 * i + s
        strand_seq = q if i % 2 == 0 else rc
        # N at window offset o inside word 33 of the wave (base 1056 onwards)
        choices = [o for o in range(1056 - s, L) if strand_seq[o] != ord("G")]
        o = rng.choice(choices)
        w = bytearray(strand_seq)
        subs = rng.sample([x for x in range(L) if x != o], 16)
        for x in subs:
            w[x] = rng.choice([b for b in b"ACGT" if b != w[x]])
        w[o] = ord("N")
        contig[start:start + L] = w
    k = 16 if policy == 0 else 17
    want = orc.scan([q], [bytes(contig)], [k], policy=policy)
    assert len(want) >= 8
    vs = [v for v in range(ifa.ifa_variant_count())
          if ifa.ifa_variant_info(v)["encoding"] in (2, 3)]
    assert vs
    for v in vs:
        say(f"N in word 33: variant {v} policy {policy}")
        with ifa.Scanner(n_policy=policy) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries([q], [k])
            assert ifa.ifa_query_partition(s.ctx) == (2, 2)
            s.scan_chunk([bytes(contig)])
            assert_same(s.collect(), want, f"variant {v}")


@pytest.mark.parametrize("policy", [0, 1])
def test_longest_query_inside_an_n_run(ifa, orc, policy):
    """The longest query (255 bases) over a run of 300 Ns: windows inside the
    run have n_ref = 255, which must come back whole in the record and in the
    digest. N_SEPARATE with maxN = 255 reports them (m = 0); N_AS_MISMATCH
    with maxSubs = 255 reports them with m = 255."""
    rng = random.Random(255)
    L = 255
    q = rand_dna(rng, L)
    contig = rand_dna(rng, 700) + b"N" * 300 + rand_dna(rng, 700)
    ks, mn = [L], [L]
    say(f"L=255 over 300 Ns, policy {policy}")
    want, cnt, dig = orc.scan([q], [contig], ks, mn, policy=policy, stats=True)
    assert (want["n_ref"] == 255).sum() == 2 * 46
    got = gpu_scan(ifa, [q], [contig], ks, mn, n_policy=policy)
    assert_same(got, want, "L=255 in an N run")
    with ifa.Scanner(n_policy=policy, sink=1) as s:
        s.load_queries([q], ks, mn)
        s.scan_chunk([contig])
        gc, gd = s.query_stats()
    assert np.array_equal(gc, cnt) and np.array_equal(gd, dig)


def test_filter_launch_split_past_65535_batches(ifa, orc):
    """The matrix-core filters take one batch of 32 sparse strands per grid
    row, and a launch holds at most 65,535 rows: 1,050,000 queries of 32 bases
    (2.1 M strands, 65,625 batches) make the host launch the filter in two
    parts, the second starting at batch 65,535. Copies of queries from both
    parts are planted in a small reference; the three-class and four-class
    filters must both give the oracle's hits."""
    n = 1_050_000
    L, k = 32, 2
    rng = np.random.default_rng(65535)
    codes = np.frombuffer(b"ACGT", dtype=np.uint8)[rng.integers(0, 4, size=(n, L))]
    qs = [codes[i].tobytes() for i in range(n)]
    r = random.Random(65535)
    contigs = [bytearray(rand_dna(r, 700)) for _ in range(2)]
    planted = [0, 1, 31, 500_000, 1_048_560, 1_049_000] + list(range(n - 8, n))
    for i, j in enumerate(planted):
        c = contigs[i % 2]
        p = 40 + 90 * (i // 2)
        src = bytearray(qs[j] if i % 3 else qs[j].translate(COMP)[::-1])
        for x in r.sample(range(L), i % 3):
            src[x] = r.choice([b for b in b"ACGT" if b != src[x]])
        c[p:p + L] = src
    contigs = [bytes(c) for c in contigs]
    ks = [k] * n
    say(f"launch split: {n} queries, oracle")
    want = orc.scan(qs, contigs, ks)
    assert set(planted) <= set(want["query"].tolist())
    for enc in (2, 1):
        v = next(v for v in range(ifa.ifa_variant_count())
                 if ifa.ifa_variant_info(v)["encoding"] == enc)
        say(f"launch split: variant {v} (encoding {enc})")
        with ifa.Scanner(chunk_bases=8192) as s:
            ifa.ifa_set_variant(s.ctx, v)
            s.load_queries(qs, ks)
            assert ifa.ifa_query_partition(s.ctx) == (2 * n, 2 * n)
            s.scan_chunk(contigs)
            assert_same(s.collect(), want, f"variant {v}")


@pytest.mark.parametrize("sink", [0, 1])
def test_dense_strands_on_matrix_cores(ifa, orc, sink):
    """Dense strands of at most 32 bases with a random-window hit rate of at
    most 5 % are counted on the matrix cores on clean waves (no N or contig
    end among the words their windows read) and by the VALU kernels
    elsewhere; the other dense strands always by the VALU kernels, which run
    the two groups (each by L descending) in launches of their own. Short
    high-threshold queries (hit rates from 1e-4 to ~1) against contigs with N
    runs and many contig ends, in small chunks (carried prefixes), records
    with a small hit buffer (re-scans) and count+digest: every three-class
    variant and a VALU variant equal the oracle. A-rich and T-rich queries
    give strands whose required count L - k - nA is negative (the three-class
    value of a window is negative where the reference misses query A bases)."""
    rng = random.Random(4422)
    contigs = []
    for i in range(10):
        n = rng.choice([900, 5000, 33_000, 70_000])
        c = bytearray(rand_dna(rng, n))
        for _ in range(rng.randint(0, 3)):
            p = rng.randrange(0, n - 1)
            c[p:p + rng.randint(1, 120)] = b"N" * len(c[p:p + 120])
        contigs.append(bytes(c[:n]))
    qs, ks = [], []
    for L, k in ((18, 16), (18, 12), (20, 10), (24, 12), (24, 9), (28, 14), (31, 15),
                 (32, 16), (32, 13), (36, 16), (37, 17), (19, 11), (22, 8), (26, 10)):
        for _ in range(3):
            qs.append(rand_dna(rng, L, b"ACGT" if rng.random() < 0.9 else b"ACGTN"))
            ks.append(k)
    # matrix-core strands (hit rate at most 5 %) with more A bases than L - k
    for L, k, base in ((20, 11, b"A"), (26, 15, b"A"), (18, 9, b"T"), (28, 15, b"T")):
        for _ in range(2):
            q = bytearray(rand_dna(rng, L))
            for i in rng.sample(range(L), L - k + 2):
                q[i] = base[0]
            qs.append(bytes(q))
            ks.append(k)
    if sink == 0:
        want = orc.scan(qs, contigs, ks)
    else:
        _, cnt, dig = orc.scan(qs, contigs, ks, stats=True, records=False)
    vs = [v for v in range(ifa.ifa_variant_count()) if ifa.ifa_variant_info(v)["encoding"] == 3]
    assert vs, "no variant with dense strands on the matrix cores"
    vs.append(next(v for v in range(ifa.ifa_variant_count())
                   if ifa.ifa_variant_info(v)["encoding"] == 2))
    vs.append(next(v for v in range(ifa.ifa_variant_count())
                   if ifa.ifa_variant_info(v)["encoding"] == 0
                   and ifa.ifa_variant_info(v)["windows_per_lane"] == 16))
    for v in vs:
        for chunk, hcap in ((1 << 20, 0), (1 << 16, 20_000)):
            say(f"dense on matrix cores: variant {v} sink {sink} chunk {chunk} hcap {hcap}")
            with ifa.Scanner(chunk_bases=chunk, sink=sink,
                             hit_capacity=hcap if sink == 0 else 0) as s:
                ifa.ifa_set_variant(s.ctx, v)
                s.load_queries(qs, ks)
                n_strands, n_filtered = ifa.ifa_query_partition(s.ctx)
                assert n_filtered < n_strands
                s.scan_chunk(contigs)
                if sink == 0:
                    assert_same(s.collect(), want, f"variant {v} chunk {chunk}")
                else:
                    gc, gd = s.query_stats()
                    assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), f"variant {v}"


def test_variant_chosen_after_loading_builds_its_operands(ifa, orc):
    """The query tables carry the matrix-filter operands of the variant in use
    when the queries are loaded; a variant chosen afterwards builds its own
    (four-class, three-class, three-class with dense strands on the matrix
    cores) on its first scan. One load, then every encoding in turn and back
    to the first, each scan equal to the oracle."""
    rng = random.Random(2718)
    contigs = []
    for _ in range(6):
        n = rng.choice([4000, 30_000, 90_000])
        c = bytearray(rand_dna(rng, n))
        p, r = rng.randrange(0, n - 200), rng.randint(1, 150)
        c[p:p + r] = b"N" * r
        contigs.append(bytes(c))
    qs, ks = [], []
    for L, k in ((34, 3), (40, 5), (30, 2), (64, 9), (20, 9), (24, 11), (31, 14), (50, 14)):
        for _ in range(3):
            qs.append(rand_dna(rng, L))
            ks.append(k)
    want = orc.scan(qs, contigs, ks)
    by_enc = {}
    for v in range(ifa.ifa_variant_count()):
        by_enc.setdefault(ifa.ifa_variant_info(v)["encoding"], v)
    order = [by_enc[e] for e in sorted(by_enc)]
    order += [order[0], order[-1], by_enc.get(2, order[0])]
    with ifa.Scanner(chunk_bases=1 << 18) as s:
        ifa.ifa_set_variant(s.ctx, order[0])
        s.load_queries(qs, ks)
        for v in order:
            say(f"variant {v} (encoding {ifa.ifa_variant_info(v)['encoding']}) after loading")
            ifa.ifa_set_variant(s.ctx, v)
            first = s.scan_chunk(contigs)   # contigs take new ordinals each call
            got = s.collect()
            got["contig"] -= first
            assert_same(got, want, f"variant {v} chosen after loading")


@pytest.mark.parametrize("sink", [0, 1])
def test_half_step_tiles_for_exact_match_queries(ifa, orc, sink):
    """Column tiles whose strands all have maxSubs 0 (and enough length) run
    the first K step of the three-class contraction alone, testing the
    window at shift r of each 8-window group on its first 16 - r bases.
    Planted exact copies at every shift and around wave and chunk edges, N
    runs, queries with an N, and sets mixing maxSubs 0 with maxSubs 1-2 (so
    that some tiles run half and others both steps) must equal the oracle
    for every three-class variant."""
    rng = random.Random(1616)
    # L 8 stays a two-step tile (its 8 bases pass too often); from L 12 on the
    # shifts whose 16 - r bases exceed L test the whole query
    lens = [8, 12, 13, 16, 17, 20, 24, 31, 32, 33, 40, 48, 64]
    qs = [rand_dna(rng, L) for L in lens for _ in range(2)]
    qs.append(rand_dna(rng, 30)[:12] + b"N" + rand_dna(rng, 17))
    contigs = []
    for i in range(8):
        n = rng.choice([3000, 40_000, 70_000])
        c = bytearray(rand_dna(rng, n))
        for _ in range(rng.randint(0, 2)):
            p, r = rng.randrange(0, n - 300), rng.randint(1, 200)
            c[p:p + r] = b"N" * r
        # exact copies (or reverse complements) at every offset mod 8 and
        # around 1024-base wave edges
        for j in range(12):
            q = qs[rng.randrange(len(qs))]
            if rng.random() < 0.5:
                q = q.translate(COMP)[::-1]
            p = rng.choice([1024 * rng.randrange(1, n // 1024 or 2) - rng.randrange(0, 40),
                            rng.randrange(0, n - len(q))])
            p = max(0, min(p, n - len(q)))
            c[p:p + len(q)] = q
        contigs.append(bytes(c))
    sets = {"all maxSubs 0": [0] * len(qs),
            "mixed": [rng.choice([0, 0, 0, 1, 2]) for _ in qs]}
    vs = [v for v in range(ifa.ifa_variant_count()) if ifa.ifa_variant_info(v)["encoding"] >= 2]
    for name, ks in sets.items():
        if sink == 0:
            want = orc.scan(qs, contigs, ks)
        else:
            _, cnt, dig = orc.scan(qs, contigs, ks, stats=True, records=False)
        for v in vs:
            say(f"half-step tiles: {name}, variant {v}, sink {sink}")
            with ifa.Scanner(chunk_bases=1 << 16, sink=sink) as s:
                ifa.ifa_set_variant(s.ctx, v)
                s.load_queries(qs, ks)
                s.scan_chunk(contigs)
                if sink == 0:
                    assert_same(s.collect(), want, f"{name} variant {v}")
                else:
                    gc, gd = s.query_stats()
                    assert np.array_equal(gc, cnt) and np.array_equal(gd, dig), \
                        f"{name} variant {v} stats"


def test_graphs_switched_off_and_on_time_every_eager_pass(ifa, orc):
    """Replayed passes are timed as a whole; turning graph capture off makes
    every later pass eager, with its kernels timed one by one, and on again
    resumes the replays. Results stay those of the oracle throughout."""
    import synth
    spec = synth.c2_spec(seed=77, total=2_000_000)
    ref = synth.gen_reference(spec)
    rng = random.Random(77)
    qs = [rand_dna(rng, rng.choice([28, 32, 36])) for _ in range(6)]
    ks = [rng.randint(0, 4) for _ in qs]
    want = orc.scan(qs, ref, ks)
    with ifa.Scanner(chunk_bases=1 << 20) as s:
        s.ref_load(ref)
        s.load_queries(qs, ks)
        _, chunks = ifa.ifa_ref_info(s.ctx)
        for i in range(3):
            s.scan_resident()
            assert_same(s.collect(), want, f"graph pass {i}")
        st = s.stats()
        assert st["graph_launches"] > 0
        assert st["timed_passes"] == st["kernel_launches"] - st["graph_launches"]
        ifa.ifa_set_graphs(s.ctx, False)
        ifa.ifa_reset_stats(s.ctx)
        for i in range(2):
            s.scan_resident()
            assert_same(s.collect(), want, f"eager pass {i}")
        st = s.stats()
        assert st["graph_launches"] == 0 and st["timed_passes"] == st["kernel_launches"] == 2 * chunks
        assert st["timed_filter_passes"] == 2 * chunks and st["filter_ms"] > 0
        ifa.ifa_set_graphs(s.ctx, True)
        ifa.ifa_reset_stats(s.ctx)
        s.scan_resident()
        assert_same(s.collect(), want, "graphs on again")
        assert s.stats()["graph_launches"] > 0
