"""The seeded generator: determinism, independent regeneration of any range,
and the shapes and rates each workload recipe promises."""
import math

import numpy as np


def test_reference_is_deterministic(synth_mod):
    spec = synth_mod.c2_spec(seed=42, total=3_000_000)
    a = synth_mod.gen_reference(spec, threads=1)
    b = synth_mod.gen_reference(spec, threads=5)
    assert np.array_equal(a.lens, b.lens)
    assert np.array_equal(a.buf, b.buf)
    assert a.total == 3_000_000


def test_any_range_regenerates_independently(synth_mod):
    spec = synth_mod.c2_spec(seed=8, total=2_000_000)
    spec.n_param = 5e-3          # many N runs so runs crossing blocks are exercised
    ref = synth_mod.gen_reference(spec)
    rng = np.random.default_rng(0)
    for _ in range(50):
        c = int(rng.integers(0, ref.n_contigs))
        n = int(ref.lens[c])
        x0 = int(rng.integers(0, n))
        m = int(rng.integers(1, min(20000, n - x0) + 1))
        part = synth_mod.fill_range(spec, c, n, float(ref.gcs[c]), x0, m)
        assert np.array_equal(part, ref.contig(c)[x0:x0 + m])


def test_c2_shape(synth_mod):
    spec = synth_mod.c2_spec(seed=2, total=200_000_000)
    ref = synth_mod.gen_reference(spec)
    assert ref.total == 200_000_000
    assert int(ref.lens[:-1].min()) >= 1000
    frac_n = float((ref.buf == ord("N")).mean())
    assert 0.5e-4 < frac_n < 2e-4
    gc = ((ref.buf == ord("G")) | (ref.buf == ord("C"))).mean()
    assert 0.35 < gc < 0.65
    # per-contig GC follows the contig's drawn value
    for c in range(min(ref.n_contigs, 5)):
        s = ref.contig(c)
        if s.size > 200_000:
            g = ((s == ord("G")) | (s == ord("C"))).mean()
            assert abs(g - ref.gcs[c]) < 0.01


def test_c1_shape(synth_mod):
    w = synth_mod.c1_tiny()
    assert w.ref.n_contigs == 10 and w.ref.total == 1_000_000
    assert len(w.queries) == 1 and len(w.queries[0]) == 32
    assert len(w.plants) == 20 and sum(p.strand for p in w.plants) == 10
    assert all(0 <= p.subs <= 3 for p in w.plants)
    assert 0.0008 < float((w.ref.buf == ord("N")).mean()) < 0.0012


def test_c4_contig_lengths_in_range(synth_mod):
    spec = synth_mod.c4_spec(seed=4, total=2_000_000_000)
    lens = synth_mod.contig_lengths(spec)
    assert int(lens.sum()) == 2_000_000_000
    assert int(lens[:-1].min()) >= 1_000_000 and int(lens.max()) <= 10_000_000
    med = float(np.median(lens))
    assert abs(math.log(med / (math.sqrt(10) * 1e6))) < 0.2


def test_queries_and_trace(synth_mod):
    qs = synth_mod.gen_queries(3, 2000, 18, 50)
    lens = [len(q) for q in qs]
    assert min(lens) == 18 and max(lens) == 50
    assert set(b"".join(qs)) <= set(b"ACGT")
    tr = synth_mod.c5_trace(seed=5, n_requests=50)
    assert len(tr) == 50
    for t, q, k in tr:
        assert 1 <= len(q) <= 1000
        assert all(0 <= kk <= len(qq) // 4 for qq, kk in zip(q, k))



def test_vector_and_scalar_generators_agree(synth_mod):
    """The AVX2 base generator writes exactly the scalar generator's bytes,
    for GC levels from 0 to 1 and for ranges that start and end inside a
    draw or a block."""
    import numpy as np
    spec = synth_mod.c4_spec(seed=11, total=3_000_000)
    cases = [(0, 100_000, gc, x0, n) for gc in (0.0, 0.3, 0.5, 0.77, 0.999, 1.0)
             for (x0, n) in ((0, 100_000), (3, 9_001), (4095, 8_200), (12_345, 67))]
    got = [synth_mod.fill_range(spec, c, clen, gc, x0, n) for c, clen, gc, x0, n in cases]
    ref_v = synth_mod.gen_reference(spec)
    synth_mod.set_simd(False)
    try:
        want = [synth_mod.fill_range(spec, c, clen, gc, x0, n) for c, clen, gc, x0, n in cases]
        ref_s = synth_mod.gen_reference(spec)
    finally:
        synth_mod.set_simd(True)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert np.array_equal(ref_v.buf, ref_s.buf)


def test_packed_planes_hold_the_same_bases(synth_mod):
    """fill_packed writes the bases fill_contigs writes, as the 2-bit code
    planes of a packed chunk (hi = bit 2, lo = bit 1 of the ASCII letter),
    with and without the AVX2 path, for contigs at unaligned offsets."""
    import numpy as np
    spec = synth_mod.c4_spec(total=30_000_000)
    lens = np.array([5, 31, 32, 33, 4095, 4096, 4097, 100_003, 1_000_000, 77], dtype=np.uint64)
    gcs = synth_mod.contig_gc(spec, 0, len(lens))
    offs = np.zeros(len(lens), dtype=np.uint64)
    offs[1:] = np.cumsum(lens)[:-1]
    total = int(lens.sum())
    buf = np.empty(total, dtype=np.uint8)
    synth_mod.fill_contigs(spec, 3, lens, gcs, buf, offs)
    words = (total + 31) // 32
    bits = np.zeros(words * 32, dtype=np.uint8)
    want = []
    for b in (2, 1):
        bits[:total] = (buf >> b) & 1
        want.append(np.packbits(bits.reshape(-1, 8), axis=1, bitorder="little")
                    .reshape(-1).view(np.uint32))
    for simd in (True, False):
        synth_mod.set_simd(simd)
        hi = np.full(words, 0xDEADBEEF, dtype=np.uint32)
        lo = np.full(words, 0xDEADBEEF, dtype=np.uint32)
        assert synth_mod.fill_packed(spec, 3, lens, gcs, hi, lo, threads=3) == total
        assert np.array_equal(hi, want[0]) and np.array_equal(lo, want[1]), simd
    synth_mod.set_simd(True)
