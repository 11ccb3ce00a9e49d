"""Oracle for the brute-force gapless scan -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check in __graft_entry__ and the CPU-baseline leg of
bench.py may import this package. The product path (the HIP library and its
binding) never imports it and shares no code with it.

Two independent implementations of the same plain definition:
  * `scan` -- the C oracle in ifa_oracle.c (multi-threaded, byte compare);
  * `brute_scan` -- a numpy brute force over every window, for tiny inputs.
The definition and every reading of the paper it takes are stated at the top
of ifa_oracle.c.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

HIT_DTYPE = np.dtype([("query", "<u4"), ("contig", "<u4"), ("pos", "<i4"), ("strand", "u1"),
                      ("n_ref", "u1"), ("mismatches", "<u2")])
assert HIT_DTYPE.itemsize == 16

N_SEPARATE, N_AS_MISMATCH = 0, 1

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        i64 = ctypes.c_int64
        L.orc_scan.argtypes = [u32, vp, vp, vp, vp, u32, vp, vp, u32, u32, u32, ctypes.c_int,
                               vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp),
                               ctypes.POINTER(u64), vp, vp]
        L.orc_scan.restype = ctypes.c_int
        L.orc_free.argtypes = [vp]
        L.orc_mix64.argtypes = [u64]
        L.orc_mix64.restype = u64
        L.orc_hit_hash.argtypes = [u32, i32, u32, u32, u32]
        L.orc_hit_hash.restype = u64
        L.orc_eval_window.argtypes = [vp, u32, i32, i32, vp, u64, i64, u32, u32, ctypes.c_int,
                                      ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.orc_eval_window.restype = ctypes.c_int
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_splitmix64.restype = u64
        L.orc_keff.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_keff.restype = ctypes.c_int
        L.orc_minhits.argtypes = [i32, i32, i32, i32, i32, u64, u64, u32]
        L.orc_minhits.restype = i64
        _lib = L
    return _lib


def _default_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _as_bytes(x) -> bytes:
    if isinstance(x, (bytes, bytearray)):
        return bytes(x)
    if isinstance(x, str):
        return x.encode()
    return np.ascontiguousarray(x, dtype=np.uint8).tobytes()


class _Contigs:
    """Keeps contig buffers alive and exposes pointer/length arrays."""

    def __init__(self, contigs):
        self.keep = []
        ptrs = []
        lens = []
        for c in contigs:
            if isinstance(c, np.ndarray):
                a = np.ascontiguousarray(c, dtype=np.uint8)
            else:
                a = np.frombuffer(_as_bytes(c), dtype=np.uint8)
            self.keep.append(a)
            ptrs.append(a.ctypes.data if a.size else 0)
            lens.append(a.size)
        n = len(ptrs)
        self.ptrs = (ctypes.c_void_p * max(n, 1))(*ptrs)
        self.lens = np.array(lens if n else [0], dtype=np.uint64)
        self.n = n


class _SeedSpec(ctypes.Structure):
    _fields_ = [("k", ctypes.c_void_p), ("thr", ctypes.c_void_p), ("mask", ctypes.c_int32),
                ("step", ctypes.c_int32)]


def scan(queries, contigs, max_subs, max_n=None, *, first_ordinal=0, strands=3,
         policy=N_SEPARATE, overhang=False, seeds=None, threads=None, records=True,
         stats=False):
    """Run the C oracle.

    queries: list of byte strings; contigs: list of byte strings / uint8 arrays
    (or a synth.Reference); max_subs: per-query ints; max_n: per-query ints or
    None (floor(L/4)); overhang: also the windows hanging off a contig end by
    at most min(maxN, L - 1) bases; seeds: indexed mode, a dict with per-query
    "k", per-query-and-strand "thr" ([[t_fwd, t_rc], ...]), "mask" and "step"
    (see indexed_params). Returns a HIT_DTYPE array in (contig, pos, strand,
    query) order; with stats=True returns (hits, counts, digests).
    """
    if hasattr(contigs, "pointer_array"):
        ptrs, lens = contigs.pointer_array()
        keep = (contigs,)
        nc = contigs.n_contigs
    else:
        C = _Contigs(contigs)
        ptrs, lens, keep, nc = C.ptrs, C.lens, (C,), C.n
    qb = [_as_bytes(q) for q in queries]
    nq = len(qb)
    qbufs = [np.frombuffer(q, dtype=np.uint8) if q else np.zeros(1, np.uint8) for q in qb]
    qptrs = (ctypes.c_void_p * max(nq, 1))(*[b.ctypes.data for b in qbufs])
    qlen = np.array([len(q) for q in qb] or [0], dtype=np.uint32)
    ks = np.array(list(max_subs) or [0], dtype=np.int32)
    mn = None if max_n is None else np.array(list(max_n) or [0], dtype=np.int32)
    counts = np.zeros(max(nq, 1), dtype=np.uint64)
    digests = np.zeros(max(nq, 1), dtype=np.uint64)
    spec = None
    if seeds is not None:
        sk = np.ascontiguousarray(list(seeds["k"]) or [1], dtype=np.int32)
        st = np.ascontiguousarray(np.asarray(seeds["thr"], dtype=np.int32).reshape(-1) if nq
                                  else [0, 0], dtype=np.int32)
        spec = _SeedSpec(sk.ctypes.data, st.ctypes.data, int(seeds.get("mask", 0)),
                         int(seeds.get("step", 1)))
    out = ctypes.c_void_p()
    n_out = ctypes.c_uint64()
    rc = lib().orc_scan(nq, qptrs, qlen.ctypes.data, ks.ctypes.data,
                        None if mn is None else mn.ctypes.data, nc, ptrs, lens.ctypes.data,
                        first_ordinal, strands, policy, 1 if overhang else 0,
                        None if spec is None else ctypes.byref(spec),
                        threads or _default_threads(),
                        1 if records else 0, ctypes.byref(out), ctypes.byref(n_out),
                        counts.ctypes.data, digests.ctypes.data)
    del keep
    if rc != 0:
        raise ValueError("oracle scan failed (bad arguments or out of memory)")
    hits = np.zeros(0, dtype=HIT_DTYPE)
    if records:
        n = n_out.value
        if n:
            buf = (ctypes.c_char * (n * 16)).from_address(out.value)
            hits = np.frombuffer(bytes(buf), dtype=HIT_DTYPE).copy()
        lib().orc_free(out)
    if stats:
        return hits, counts[:nq], digests[:nq]
    return hits


def eval_window(query, max_subs, contig, pos, strand, max_n=-1, policy=N_SEPARATE,
                overhang=False):
    """Exact (hit, mismatches, n_ref) of one window; None if it is not a
    window of the scan."""
    q = np.frombuffer(_as_bytes(query), dtype=np.uint8)
    c = contig if isinstance(contig, np.ndarray) else np.frombuffer(_as_bytes(contig), np.uint8)
    c = np.ascontiguousarray(c, dtype=np.uint8)
    m = ctypes.c_int32()
    nr = ctypes.c_int32()
    rc = lib().orc_eval_window(q.ctypes.data, len(q), max_subs, max_n, c.ctypes.data, c.size,
                               pos, strand, policy, 1 if overhang else 0, ctypes.byref(m),
                               ctypes.byref(nr))
    if rc < 0:
        return None
    return bool(rc), m.value, nr.value


def mix64(z: int) -> int:
    return int(lib().orc_mix64(z))


def splitmix64(seed: int, n: int) -> int:
    """Draw n (0-based) of the SplitMix64 stream with this seed."""
    return int(lib().orc_splitmix64(seed, n))


def keff(k: int, mask: int = 0, step: int = 1) -> int:
    return int(lib().orc_keff(k, mask, step))


def minhits(valid, subs, k, mask=0, step=1, iters=200_000, seed=1, ppm=999_000) -> int:
    """MinHits for a query with `valid` seeds (see ifa_oracle.c); may be <= 0."""
    r = int(lib().orc_minhits(valid, subs, k, mask, step, iters, seed, ppm))
    if r == -(1 << 63):
        raise ValueError("bad MinHits arguments")
    return r


# Indexed-mode defaults (Methods, "Algorithm Design"): candidate seed lengths,
# 200,000 Monte Carlo trials, 99.9 % probability.
SEED_KS = (8, 9, 10, 12, 14)


def _valid_seeds(codes, k, mask, step):
    lo = (k - mask) // 2
    n = 0
    for i in range(0, len(codes) - k + 1, step):
        if all(codes[i + t] != 4 for t in range(k) if t < lo or t >= lo + mask):
            n += 1
    return n


def indexed_params(queries, max_subs, *, ks=SEED_KS, mask=0, step=1, iters=200_000, seed=1,
                   ppm=999_000):
    """Per query: the seed length k and the per-strand seed thresholds.

    Readings of the multi-K rule (Methods, "Algorithm Design"): the longest k
    in `ks` (k <= L, k > mask) whose MinHits on the query's forward strand is
    at least 1; if none, the shortest such k; a query shorter than every k
    uses k = L. The threshold of a strand is max(1, MinHits) for its own
    valid-seed count: a window needs one error-free seed to be found at all.
    """
    out_k, out_thr = [], []
    cache = {}

    def mh(v, s, k):
        key = (v, s, k)
        if key not in cache:
            cache[key] = minhits(v, s, k, mask, step, iters, seed, ppm) if v > 0 else 0
        return cache[key]

    for q, s in zip(queries, max_subs):
        c = _CODE[np.frombuffer(_as_bytes(q), dtype=np.uint8)].tolist()
        rc = [4 if x == 4 else 3 - x for x in reversed(c)]
        L = len(c)
        s = min(int(s), L)
        if L <= mask:
            raise ValueError("a query must be longer than the seed mask")
        cand = sorted((k for k in ks if k <= L and k > mask), reverse=True) or [L]
        k = next((k for k in cand if mh(_valid_seeds(c, k, mask, step), s, k) >= 1), cand[-1])
        out_k.append(k)
        out_thr.append([max(1, mh(_valid_seeds(x, k, mask, step), s, k)) for x in (c, rc)])
    return {"k": out_k, "thr": out_thr, "mask": mask, "step": step}


def hit_hash(contig, pos, strand, mism, nref) -> int:
    return int(lib().orc_hit_hash(contig, pos, strand, mism, nref))


# ---------------------------------------------------------------------------
# numpy brute force (tiny inputs only)
# ---------------------------------------------------------------------------

_CODE = np.full(256, 4, dtype=np.int8)
for _i, _ch in enumerate(b"ACGT"):
    _CODE[_ch] = _i
    _CODE[_ch + 32] = _i


def brute_scan(queries, contigs, max_subs, max_n=None, *, first_ordinal=0, strands=3,
               policy=N_SEPARATE, overhang=False):
    """Every window of every contig, every query and strand, by whole-array
    comparison. Same output format and order as `scan`. With overhang the
    contig is first padded with L - 1 N codes on each side and a window may
    hold at most min(maxN, L - 1) of them."""
    rows = []
    for ci, c in enumerate(contigs):
        r0 = _CODE[np.frombuffer(_as_bytes(c), dtype=np.uint8)]
        n = r0.size
        for j, qq in enumerate(queries):
            q = _CODE[np.frombuffer(_as_bytes(qq), dtype=np.uint8)]
            L = q.size
            mn = L // 4 if max_n is None else max_n[j]
            K = min(max_subs[j], L)
            M = min(mn, L)
            pad = L - 1 if overhang else 0
            r = np.concatenate([np.full(pad, 4, np.int8), r0, np.full(pad, 4, np.int8)])
            off_contig = np.concatenate([np.ones(pad, bool), np.zeros(n, bool),
                                         np.ones(pad, bool)])
            if L > r.size:
                continue
            W = np.lib.stride_tricks.sliding_window_view(r, L)        # (n+2pad-L+1, L)
            off = np.lib.stride_tricks.sliding_window_view(off_contig, L).sum(axis=1)
            inside = off <= min(mn, L - 1)
            rN = W == 4
            nref = rN.sum(axis=1)
            qrc = np.where(q[::-1] == 4, 4, 3 - q[::-1])
            for s, qs in ((0, q), (1, qrc)):
                if not strands & (1 << s):
                    continue
                if policy == N_SEPARATE:
                    m = ((W != qs[None, :]) & ~rN).sum(axis=1)
                    ok = (m <= K) & (nref <= M)
                else:
                    m = ((W != qs[None, :]) | rN | (qs[None, :] == 4)).sum(axis=1)
                    ok = m <= K
                ok &= inside if overhang else off == 0
                for p in np.nonzero(ok)[0]:
                    rows.append((j, first_ordinal + ci, int(p) - pad, s, int(nref[p]),
                                 int(m[p])))
    out = np.array(rows, dtype=HIT_DTYPE) if rows else np.zeros(0, dtype=HIT_DTYPE)
    return sort_hits(out)


def sort_hits(h: np.ndarray) -> np.ndarray:
    """Canonical order: (contig, pos, strand, query)."""
    if h.size == 0:
        return h
    idx = np.lexsort((h["query"], h["strand"], h["pos"], h["contig"]))
    return h[idx]
