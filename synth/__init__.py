"""Seeded synthetic inputs for the gapless scan: reference contigs, query sets,
planted copies and serving traces.

This package only generates inputs. It computes nothing the aligner computes;
both the HIP path and the oracle receive its output as ASCII bytes. Bases come
from the counter-based generator in synth.c, so a contig range can be rebuilt
from the seed alone. Small per-query draws (thresholds, planting, arrival
times) use numpy's PCG64 seeded from the same seed.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        u64, i64, u32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double
        vp = ctypes.c_void_p
        L.synth_splitmix64.argtypes = [u64, u64, vp]
        L.synth_contig_lengths.argtypes = [u64, ctypes.c_int, u64, u64, dbl, dbl, u64, u64, u64,
                                           vp, i64]
        L.synth_contig_lengths.restype = i64
        L.synth_contig_gc.argtypes = [u64, u64, u64, dbl, dbl, vp]
        L.synth_fill.argtypes = [u64, ctypes.c_int, dbl, u32, u32, u64, u64, dbl, u64, u64, vp]
        L.synth_fill_many.argtypes = [u64, ctypes.c_int, dbl, u32, u32, u64, u64, vp, vp, vp, vp,
                                      ctypes.c_int]
        L.synth_fill_many.restype = ctypes.c_int
        L.synth_fill_packed.argtypes = [u64, u64, u64, vp, vp, vp, vp, ctypes.c_int]
        L.synth_fill_packed.restype = ctypes.c_int
        L.synth_queries.argtypes = [u64, u64, u64, u32, u32, vp, u64, vp]
        L.synth_set_simd.argtypes = [ctypes.c_int]
        L.synth_set_simd.restype = None
        _lib = L
    return _lib


def set_simd(on: bool):
    """Use (default) or bypass the AVX2 base generator; output is identical."""
    lib().synth_set_simd(1 if on else 0)


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().synth_splitmix64(seed, n, out.ctypes.data)
    return out


def default_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


# --------------------------------------------------------------------------
# reference
# --------------------------------------------------------------------------

N_NONE, N_IID, N_RUNS = 0, 1, 2


@dataclass
class RefSpec:
    """How a synthetic reference is drawn."""
    seed: int
    total: int = 0                 # total bases (length modes 1 and 2)
    length_mode: int = 1           # 0 fixed, 1 lognormal with floor, 2 lognormal resampled
    n_fixed: int = 0
    fixed_len: int = 0
    median: float = 3e6
    sigma: float = 1.0
    min_len: int = 1000
    max_len: int = 0
    gc_lo: float = 0.5
    gc_hi: float = 0.5
    n_mode: int = N_NONE
    n_param: float = 0.0
    run_min: int = 10
    run_max: int = 190


@dataclass
class Reference:
    """Contigs stored back to back in one uint8 buffer."""
    buf: np.ndarray                # uint8, ASCII bases
    offs: np.ndarray               # uint64 start of each contig in buf
    lens: np.ndarray               # uint64 length of each contig
    gcs: np.ndarray = field(default=None)

    @property
    def n_contigs(self) -> int:
        return len(self.lens)

    @property
    def total(self) -> int:
        return int(self.lens.sum())

    def contig(self, i: int) -> np.ndarray:
        o = int(self.offs[i])
        return self.buf[o:o + int(self.lens[i])]

    def contig_bytes(self, i: int) -> bytes:
        return self.contig(i).tobytes()

    def pointer_array(self):
        """(ctypes array of uint8*, numpy uint64 lengths) over the contigs."""
        base = self.buf.ctypes.data
        ptrs = (ctypes.c_void_p * self.n_contigs)(*[base + int(o) for o in self.offs])
        return ptrs, np.ascontiguousarray(self.lens, dtype=np.uint64)

    def subset(self, idx) -> "Reference":
        """A new Reference holding copies of the listed contigs (in that order)."""
        idx = list(idx)
        lens = np.array([int(self.lens[i]) for i in idx], dtype=np.uint64)
        offs = np.zeros(len(idx), dtype=np.uint64)
        if len(idx) > 1:
            offs[1:] = np.cumsum(lens)[:-1]
        buf = np.empty(int(lens.sum()), dtype=np.uint8)
        for j, i in enumerate(idx):
            buf[int(offs[j]):int(offs[j]) + int(lens[j])] = self.contig(i)
        gcs = None if self.gcs is None else np.array([self.gcs[i] for i in idx])
        return Reference(buf, offs, lens, gcs)


def contig_lengths(spec: RefSpec) -> np.ndarray:
    if spec.length_mode == 0:
        cap = spec.n_fixed
    else:
        # every contig but the last is at least min_len long
        cap = spec.total // max(1, spec.min_len) + 2
    out = np.zeros(max(cap, 1), dtype=np.uint64)
    n = lib().synth_contig_lengths(spec.seed, spec.length_mode, spec.n_fixed, spec.fixed_len,
                                   spec.median, spec.sigma, spec.min_len, spec.max_len,
                                   spec.total, out.ctypes.data, len(out))
    if n < 0:
        raise RuntimeError("contig table capacity too small")
    return out[:n].copy()


def contig_gc(spec: RefSpec, first: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float64)
    lib().synth_contig_gc(spec.seed, first, n, spec.gc_lo, spec.gc_hi, out.ctypes.data)
    return out


def fill_contigs(spec: RefSpec, first_contig: int, lens: np.ndarray, gcs: np.ndarray,
                 out: np.ndarray, offs: np.ndarray, threads: int | None = None):
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    gcs = np.ascontiguousarray(gcs, dtype=np.float64)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    assert out.dtype == np.uint8 and out.flags.c_contiguous
    if len(lens):
        assert int(offs[-1]) + int(lens[-1]) <= out.size
    rc = lib().synth_fill_many(spec.seed, spec.n_mode, spec.n_param, spec.run_min, spec.run_max,
                               first_contig, len(lens), lens.ctypes.data, gcs.ctypes.data,
                               out.ctypes.data, offs.ctypes.data, threads or default_threads())
    if rc != 0:
        raise MemoryError("synth_fill_many failed")


def fill_packed(spec: RefSpec, first_contig: int, lens: np.ndarray, gcs: np.ndarray,
                hi: np.ndarray, lo: np.ndarray, threads: int | None = None) -> int:
    """The bases fill_contigs writes, as the two 2-bit code planes of a packed
    chunk (contigs back to back from base 0; A=00 C=01 G=11 T=10 as hi, lo
    bits); references without N only. hi / lo need ceil(total / 32) uint32
    words each. Returns the total bases."""
    assert spec.n_mode == N_NONE, "packed output covers references without N"
    lens = np.ascontiguousarray(lens, dtype=np.uint64)
    gcs = np.ascontiguousarray(gcs, dtype=np.float64)
    total = int(lens.sum())
    words = (total + 31) // 32
    assert hi.dtype == np.uint32 and lo.dtype == np.uint32
    assert hi.size >= words and lo.size >= words and hi.flags.c_contiguous and lo.flags.c_contiguous
    rc = lib().synth_fill_packed(spec.seed, first_contig, len(lens), lens.ctypes.data,
                                 gcs.ctypes.data, hi.ctypes.data, lo.ctypes.data,
                                 threads or default_threads())
    if rc != 0:
        raise MemoryError("synth_fill_packed failed")
    return total


def gen_reference(spec: RefSpec, threads: int | None = None) -> Reference:
    lens = contig_lengths(spec)
    gcs = contig_gc(spec, 0, len(lens))
    offs = np.zeros(len(lens), dtype=np.uint64)
    if len(lens) > 1:
        offs[1:] = np.cumsum(lens)[:-1]
    buf = np.empty(int(lens.sum()), dtype=np.uint8)
    fill_contigs(spec, 0, lens, gcs, buf, offs, threads)
    return Reference(buf, offs, lens, gcs)


def fill_range(spec: RefSpec, contig: int, clen: int, gc: float, x0: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint8)
    lib().synth_fill(spec.seed, spec.n_mode, spec.n_param, spec.run_min, spec.run_max,
                     contig, clen, gc, x0, n, out.ctypes.data)
    return out


# --------------------------------------------------------------------------
# queries
# --------------------------------------------------------------------------

def gen_queries(seed: int, n: int, lmin: int, lmax: int, tag: int = 0) -> list[bytes]:
    stride = max(lmax, 1)
    buf = np.zeros(max(n, 1) * stride, dtype=np.uint8)
    lens = np.zeros(max(n, 1), dtype=np.uint32)
    if n:
        lib().synth_queries(seed, tag, n, lmin, lmax, buf.ctypes.data, stride, lens.ctypes.data)
    return [buf[i * stride:i * stride + int(lens[i])].tobytes() for i in range(n)]


# --------------------------------------------------------------------------
# planting
# --------------------------------------------------------------------------

_COMP = bytes.maketrans(b"ACGT", b"TGCA")
_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


@dataclass
class Plant:
    query: int
    contig: int
    pos: int
    strand: int      # 0 forward copy, 1 reverse-complement copy
    subs: int        # number of substituted positions


def sample_reads(ref: Reference, n: int, L: int, subs: int, seed: int):
    """n reads of L bases cut from uniformly random in-contig positions that
    hold only A/C/G/T, each with exactly `subs` substitutions at distinct
    positions (new base uniform among the other three), reverse-complemented
    with probability 1/2. Returns (reads, origins) with origins an (n, 3)
    int64 array of (contig, pos, strand)."""
    rng = np.random.Generator(np.random.PCG64([seed, 104729, L, subs]))
    offs = ref.offs.astype(np.int64)
    ends = offs + ref.lens.astype(np.int64)
    total = int(ends[-1])
    acgt = np.zeros(256, dtype=bool)
    acgt[list(b"ACGT")] = True
    got_g = np.zeros(0, dtype=np.int64)
    while got_g.size < n:
        g = rng.integers(0, total - L + 1, size=2 * (n - got_g.size) + 16)
        c = np.searchsorted(offs, g, side="right") - 1
        ok = g + L <= ends[c]
        g = g[ok]
        win = ref.buf[g[:, None] + np.arange(L)[None, :]]
        g = g[acgt[win].all(axis=1)]
        got_g = np.concatenate([got_g, g])[:n]
    c = np.searchsorted(offs, got_g, side="right") - 1
    reads = ref.buf[got_g[:, None] + np.arange(L)[None, :]].copy()
    if subs > 0:
        where = np.argsort(rng.random((n, L)), axis=1)[:, :subs]
        code = np.full(256, 0, dtype=np.uint8)
        code[list(b"ACGT")] = np.arange(4, dtype=np.uint8)
        rows = np.arange(n)[:, None]
        old = code[reads[rows, where]]
        new = (old + rng.integers(1, 4, size=(n, subs))) % 4
        reads[rows, where] = np.frombuffer(b"ACGT", dtype=np.uint8)[new]
    strand = (rng.random(n) < 0.5).astype(np.int64)
    comp = np.arange(256, dtype=np.uint8)
    comp[list(b"ACGT")] = list(b"TGCA")
    rc = comp[reads[:, ::-1]]
    reads = np.where(strand[:, None] == 1, rc, reads)
    origins = np.stack([c, got_g - offs[c], strand], axis=1)
    return [r.tobytes() for r in reads], origins


def plant_copies(ref: Reference, queries: list[bytes], per_query: int, max_subs: int,
                 seed: int, rc_exact_half: bool = False) -> list[Plant]:
    """Overwrite reference windows with copies of each query carrying exactly
    `subs` ~ U{0..max_subs} substitutions at distinct positions (new base
    uniform among the other three), on non-overlapping in-contig positions.
    A reverse-complement copy is written for strand 1. With rc_exact_half the
    strands are an exact 50/50 split over all copies, else each is a fair coin.
    """
    rng = np.random.Generator(np.random.PCG64([seed, 7919]))
    total_copies = per_query * len(queries)
    if rc_exact_half:
        strands = np.array([0] * (total_copies - total_copies // 2) + [1] * (total_copies // 2))
        rng.shuffle(strands)
    else:
        strands = (rng.random(total_copies) < 0.5).astype(int)
    starts = np.concatenate([[0], np.cumsum(ref.lens.astype(np.int64))])
    total = int(starts[-1])
    taken: list[tuple[int, int]] = []   # global [start, end) of placed copies
    plants = []
    t = 0
    for j, q in enumerate(queries):
        L = len(q)
        for _ in range(per_query):
            for _attempt in range(100000):
                g = int(rng.integers(0, total))
                c = int(np.searchsorted(starts, g, side="right") - 1)
                pos = g - int(starts[c])
                if pos + L > int(ref.lens[c]):
                    continue
                gs, ge = g, g + L
                if any(not (ge <= a or gs >= b) for a, b in taken):
                    continue
                break
            else:
                raise RuntimeError("could not place planted copy")
            taken.append((gs, ge))
            s = int(rng.integers(0, max_subs + 1)) if max_subs > 0 else 0
            s = min(s, L)
            arr = np.frombuffer(q, dtype=np.uint8).copy()
            where = rng.choice(L, size=s, replace=False) if s else np.zeros(0, dtype=int)
            for w in where:
                cur = int(np.nonzero(_ACGT == arr[w])[0][0])
                arr[w] = _ACGT[(cur + int(rng.integers(1, 4))) % 4]
            strand = int(strands[t])
            t += 1
            window = arr.tobytes()
            if strand == 1:
                window = window.translate(_COMP)[::-1]
            o = int(ref.offs[c]) + pos
            ref.buf[o:o + L] = np.frombuffer(window, dtype=np.uint8)
            plants.append(Plant(j, c, pos, strand, s))
    return plants


# --------------------------------------------------------------------------
# workload recipes
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ref: Reference | None
    queries: list[bytes]
    max_subs: list[int]
    plants: list[Plant] = field(default_factory=list)
    spec: RefSpec | None = None
    extra: dict = field(default_factory=dict)


def c1_tiny(seed: int = 1) -> Workload:
    """1 query of length 32; 10 contigs x 100 kbp iid uniform with each base N
    at probability 0.001; 20 planted copies with 0-3 substitutions, exactly
    half reverse-complemented; maxSubs 3."""
    spec = RefSpec(seed=seed, length_mode=0, n_fixed=10, fixed_len=100_000, gc_lo=0.5,
                   gc_hi=0.5, n_mode=N_IID, n_param=0.001)
    ref = gen_reference(spec)
    qs = gen_queries(seed, 1, 32, 32)
    plants = plant_copies(ref, qs, 20, 3, seed, rc_exact_half=True)
    return Workload("c1_tiny", ref, qs, [3], plants, spec)


def c2_spec(seed: int = 2, total: int = 4_000_000_000) -> RefSpec:
    """Paper-scale reference shape: lognormal contigs (median 3 Mbp, sigma 1,
    floor 1 kbp), per-contig GC uniform in [0.35, 0.65], N runs of length
    U{10..190} covering a 1e-4 fraction."""
    return RefSpec(seed=seed, total=total, length_mode=1, median=3e6, sigma=1.0, min_len=1000,
                   gc_lo=0.35, gc_hi=0.65, n_mode=N_RUNS, n_param=1e-4, run_min=10, run_max=190)


def c2_paper_scale(seed: int = 2, total: int = 4_000_000_000, k: int = 4,
                   plants_per_query: int | None = None, n_queries: int = 10,
                   median: float = 3e6) -> Workload:
    """10 queries of length 30-36; 1 planted copy per query per 100 Mbp with
    0-8 substitutions, strand a fair coin; maxSubs k for every query. `median`
    sets the median contig length (a fragmented assembly when small)."""
    spec = c2_spec(seed, total)
    spec.median = median
    ref = gen_reference(spec)
    qs = gen_queries(seed, n_queries, 30, 36)
    if plants_per_query is None:
        plants_per_query = max(1, total // 100_000_000)
    plants = plant_copies(ref, qs, plants_per_query, 8, seed)
    return Workload(f"c2_k{k}", ref, qs, [k] * n_queries, plants, spec)


def c3_batched(seed: int = 3, total: int = 1_000_000_000, n_queries: int = 10_000,
               median: float = 3e6) -> Workload:
    """10,000 queries, lengths U{18..50}, maxSubs U{0..16} per query; reference
    from the paper-scale generator (median contig length `median`); no planted
    copies."""
    spec = c2_spec(seed, total)
    spec.median = median
    ref = gen_reference(spec) if total > 0 else None
    qs = gen_queries(seed, n_queries, 18, 50)
    rng = np.random.Generator(np.random.PCG64([seed, 31]))
    ks = [int(x) for x in rng.integers(0, 17, size=n_queries)]
    return Workload("c3_batched", ref, qs, ks, [], spec)


def c4_spec(seed: int = 4, total: int = 100_000_000_000) -> RefSpec:
    """Bacterial-genome-like contigs: lognormal with median sqrt(10) Mbp and
    sigma ln(10)/4, redrawn until inside [1, 10] Mbp; GC uniform in
    [0.30, 0.70]; no N."""
    return RefSpec(seed=seed, total=total, length_mode=2, median=math.sqrt(10.0) * 1e6,
                   sigma=math.log(10.0) / 4, min_len=1_000_000, max_len=10_000_000,
                   gc_lo=0.30, gc_hi=0.70, n_mode=N_NONE)


def c4_queries(seed: int = 4, n: int = 100):
    qs = gen_queries(seed, n, 20, 40)
    return qs, [4] * n


def c5_spec(seed: int = 5, total: int = 16_000_000_000) -> RefSpec:
    return c2_spec(seed, total)


def c5_trace(seed: int = 5, n_requests: int = 1000, rate: float = 200.0):
    """Serving trace: Poisson arrivals at `rate` per second; request sizes
    round(exp(U(0, ln 1000))) queries; lengths U{18..150}; maxSubs per query
    U{0..floor(L/4)}. Returns a list of (arrival_s, queries, max_subs)."""
    rng = np.random.Generator(np.random.PCG64([seed, 101]))
    t = 0.0
    out = []
    for r in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        n = int(round(math.exp(rng.uniform(0.0, math.log(1000.0)))))
        n = max(1, min(1000, n))
        qs = gen_queries(seed, n, 18, 150, tag=1000 + r)
        ks = [int(rng.integers(0, len(q) // 4 + 1)) for q in qs]
        out.append((t, qs, ks))
    return out
