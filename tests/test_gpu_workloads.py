"""Parity at the workloads' own shapes, through the C ABI.

Full-size runs of the paper-scale (4 Gbp) and batched (1 Gbp) workloads are
compared per query, as hit count and digest, with fixtures the oracle wrote
(tests/golden/make_workload_goldens.py). Where no fixture exists the oracle
checks what it can afford at run time: every reported hit re-evaluated window
by window, every planted copy found, and the GPU's hits on a sample of
contigs equal to the oracle's full scan of those contigs. Smaller shapes are
compared whole.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from workload_fixtures import check_fingerprint, load_golden, records_digest  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def test_c2_full_size_every_threshold(ifa):
    """The paper-scale workload at full size (4 Gbp, 10 queries L30-36) at
    maxSubs 0, 4 and 8: per-query hit count and digest of the records sink,
    and of the count+digest sink, equal the oracle's over the whole 4 Gbp
    (every contig, including those split across device chunks), and every
    planted copy within the threshold is found."""
    import synth
    say("c2 every threshold: generating 4 Gbp")
    w = synth.c2_paper_scale(total=4_000_000_000)
    head, rows = load_golden("c2_4gbp_count_digest.txt")
    check_fingerprint(head, w.ref)
    nq = len(w.queries)
    gold = {}
    for k, j, c, d in rows:
        gold.setdefault(k, (np.zeros(nq, np.uint64), np.zeros(nq, np.uint64)))
        gold[k][0][j], gold[k][1][j] = c, d
    with ifa.Scanner() as s:
        s.ref_load(w.ref)
        for k in sorted(gold):
            say(f"  records, maxSubs {k}")
            s.load_queries(w.queries, [k] * nq)
            s.scan_resident()
            got = s.collect()
            cnt, dig = records_digest(got, nq)
            assert np.array_equal(cnt, gold[k][0]), (k, cnt, gold[k][0])
            assert np.array_equal(dig, gold[k][1]), k
            found = {(int(r["query"]), int(r["contig"]), int(r["pos"]), int(r["strand"]))
                     for r in got}
            for p in w.plants:
                if p.subs <= k:
                    assert (p.query, p.contig, p.pos, p.strand) in found
    with ifa.Scanner(sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
        s.ref_load(w.ref)
        for k in sorted(gold):
            say(f"  count+digest, maxSubs {k}")
            s.load_queries(w.queries, [k] * nq)
            s.scan_resident()
            gc, gd = s.query_stats()
            assert np.array_equal(gc, gold[k][0]) and np.array_equal(gd, gold[k][1]), k


def matrix_dense_variant(ifa):
    """The variant that counts the low-hit-rate dense strands on the matrix
    cores with 256-thread filter workgroups (the batched workload's choice
    of the autotuner when the dense kernels run beside the filter)."""
    for v in range(ifa.ifa_variant_count()):
        info = ifa.ifa_variant_info(v)
        if info["encoding"] == 3 and info["workgroup"] == 256:
            return v
    raise AssertionError("no such variant")


@pytest.mark.parametrize("kind", ["default", "matrix_dense"])
def test_c3_all_queries_10mbp_of_the_1gbp_reference(ifa, kind):
    """All 10,000 batched queries (L 18-50, maxSubs 0-16) against a 10 Mbp
    sample of whole contigs of the batched workload's 1 Gbp reference:
    per-query count and digest equal the oracle's (fixture), with the
    context's default variant and with the matrix-core dense variant."""
    import re
    import synth
    w = synth.c3_batched(total=1_000_000_000)
    head, rows = load_golden("c3_10mbp_count_digest.txt")
    check_fingerprint(head, w.ref)
    pick = [int(x) for x in re.search(r"whole contigs ([0-9,]+)", " ".join(head)).group(1).split(",")]
    sub = w.ref.subset(pick)
    say(f"c3 all queries x {sub.total / 1e6:.1f} Mbp ({len(pick)} contigs), count+digest, {kind}")
    with ifa.Scanner(sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
        if kind == "matrix_dense":
            ifa.ifa_set_variant(s.ctx, matrix_dense_variant(ifa))
        s.load_queries(w.queries, w.max_subs)
        s.scan_chunk(sub)
        gc, gd = s.query_stats()
    want_c = np.array([r[1] for r in rows], dtype=np.uint64)
    want_d = np.array([r[2] for r in rows], dtype=np.uint64)
    bad = np.nonzero((gc != want_c) | (gd != want_d))[0]
    assert len(bad) == 0, f"{len(bad)} queries differ, first {bad[:5].tolist()}"
    assert int(want_c.sum()) > 10 ** 9


@pytest.mark.parametrize("kind", ["default", "matrix_dense"])
def test_c3_stratified_queries_full_1gbp(ifa, kind):
    """100 batched queries stratified over (L, maxSubs), leaving out pairs
    expected to hit more than 1e7 times, against the whole 1 Gbp batched
    reference: per-query count and digest equal the oracle's (fixture), with
    the context's default variant and with the matrix-core dense variant."""
    import synth
    w = synth.c3_batched(total=1_000_000_000)
    head, rows = load_golden("c3_100q_1gbp_count_digest.txt")
    check_fingerprint(head, w.ref)
    idx = [r[0] for r in rows]
    qs = [w.queries[i] for i in idx]
    ks = [w.max_subs[i] for i in idx]
    assert ks == [r[1] for r in rows]
    say(f"c3 stratified: {len(qs)} queries x 1 Gbp, count+digest, {kind}")
    with ifa.Scanner(sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
        if kind == "matrix_dense":
            ifa.ifa_set_variant(s.ctx, matrix_dense_variant(ifa))
        s.ref_load(w.ref)
        s.load_queries(qs, ks)
        s.scan_resident()
        gc, gd = s.query_stats()
    assert np.array_equal(gc, np.array([r[2] for r in rows], dtype=np.uint64))
    assert np.array_equal(gd, np.array([r[3] for r in rows], dtype=np.uint64))


def test_c3_all_queries_count_digest(ifa, orc):
    """All 10,000 queries (L 18-50, maxSubs 0-16) against a 400 kbp reference from
    the paper-scale generator: per-query count and digest, bit-exact."""
    import synth
    w = synth.c3_batched(total=400_000, n_queries=10_000)
    say("c3: 10,000 queries x 400 kbp, count+digest")
    _, cnt, dig = orc.scan(w.queries, w.ref, w.max_subs, records=False, stats=True)
    with ifa.Scanner(sink=ifa.IFA_SINK_COUNT_DIGEST) as s:
        s.ref_load(w.ref)
        s.load_queries(w.queries, w.max_subs)
        n_strands, n_filtered = ifa.ifa_query_partition(s.ctx)
        assert n_strands == 20_000 and 0 < n_filtered < n_strands
        s.scan_resident()
        gc, gd = s.query_stats()
    assert np.array_equal(gc, cnt)
    assert np.array_equal(gd, dig)
    assert int(cnt.sum()) > 10_000_000


def test_c3_stratified_records(ifa, orc):
    """Records for 40 of the batched queries, stratified over (L, maxSubs) and
    leaving out the pairs expected to hit more than 1e6 times, against 60 Mbp."""
    import synth
    from scipy.stats import binom
    w = synth.c3_batched(total=60_000_000, n_queries=10_000)
    cells = {}
    for i, (q, k) in enumerate(zip(w.queries, w.max_subs)):
        L = len(q)
        if 2 * 60e6 * binom.cdf(k, L, 0.75) > 1e6:
            continue
        cells.setdefault((L // 8, k // 4), []).append(i)
    pick = [v[0] for _, v in sorted(cells.items())][:40]
    qs = [w.queries[i] for i in pick]
    ks = [w.max_subs[i] for i in pick]
    say(f"c3 stratified: {len(pick)} queries x 60 Mbp, records")
    want = orc.scan(qs, w.ref, ks)
    with ifa.Scanner() as s:
        s.load_queries(qs, ks)
        s.scan_chunk(w.ref)
        got = s.collect()
    assert np.array_equal(got, want)


def test_c4_streaming_sampled_and_constant_footprint(ifa, orc):
    """Streaming 4 Gbp of the bacterial-like generator in 1 Gbp host batches
    through the pinned double buffer; hits on a 1% sample of contigs (rebuilt
    independently from the seed) must equal the oracle's; the device footprint
    after streaming equals the footprint before."""
    import synth
    total = 4_000_000_000
    spec = synth.c4_spec(total=total)
    lens = synth.contig_lengths(spec)
    gcs = synth.contig_gc(spec, 0, len(lens))
    qs, ks = synth.c4_queries(n=100)
    say(f"c4: streaming {len(lens)} contigs")
    with ifa.Scanner() as s:
        s.load_queries(qs, ks)
        foot0 = ifa.ifa_device_footprint(s.ctx)
        first = 0
        while first < len(lens):
            last, acc = first, 0
            while last < len(lens) and acc < (1 << 30):
                acc += int(lens[last])
                last += 1
            blen = lens[first:last]
            offs = np.zeros(len(blen), dtype=np.uint64)
            offs[1:] = np.cumsum(blen)[:-1]
            buf = np.empty(int(blen.sum()), dtype=np.uint8)
            synth.fill_contigs(spec, first, blen, gcs[first:last], buf, offs)
            assert s.scan_chunk(synth.Reference(buf, offs, blen)) == first
            first = last
        got = s.collect()
        foot1 = ifa.ifa_device_footprint(s.ctx)
        st = s.stats()
    assert foot1 == foot0
    assert st["bases"] >= total
    rng = np.random.default_rng(4)
    sample = sorted(rng.choice(len(lens), size=max(1, len(lens) // 100), replace=False).tolist())
    for c in sample:
        contig = synth.fill_range(spec, c, int(lens[c]), float(gcs[c]), 0, int(lens[c]))
        want = orc.scan(qs, [contig], ks, first_ordinal=c)
        assert np.array_equal(got[got["contig"] == c], want), c
