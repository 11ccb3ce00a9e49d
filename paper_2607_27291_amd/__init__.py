"""MI355X (gfx950) brute-force gapless scan of IndelFreeAligner.

Thin ctypes binding over libifa.so: each function below marshals arguments to
the C entry point of the same name in include/ifa.h. All compute runs in the
library's HIP kernels; there is no CPU fallback, and loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import itertools
import os

import numpy as np

from . import build as _build

__all__ = [
    "IfaError", "HIT_DTYPE", "lib", "ifa_config_default", "ifa_create", "ifa_destroy",
    "ifa_load_queries", "ifa_scan_chunk", "ifa_collect_hits", "ifa_last_error",
    "ifa_query_stats", "ifa_ref_load", "ifa_scan_resident", "ifa_ref_release", "ifa_ref_info",
    "ifa_get_stats", "ifa_reset_stats", "ifa_set_graphs", "ifa_set_overlap",
    "ifa_variant_count", "ifa_variant_info",
    "ifa_set_variant", "ifa_get_variant", "ifa_autotune", "ifa_query_partition",
    "ifa_device_footprint", "ifa_server_config_default", "ifa_server_create",
    "ifa_server_destroy", "ifa_server_submit", "ifa_server_step", "ifa_server_poll",
    "ifa_server_take", "ifa_server_info", "ifa_index_params_default", "ifa_set_index_params",
    "ifa_query_seeds", "ifa_query_mode", "ifa_sam_create", "ifa_sam_destroy",
    "ifa_sam_last_error", "ifa_sam_add_contigs", "ifa_sam_header", "ifa_sam_format",
    "SamWriter", "Scanner", "Server", "collect_all",
]

IFA_ABI_VERSION = 4
IFA_MAX_QUERY_LEN = 255
IFA_N_SEPARATE, IFA_N_AS_MISMATCH = 0, 1
IFA_SINK_RECORDS, IFA_SINK_COUNT_DIGEST = 0, 1
IFA_STRAND_FWD, IFA_STRAND_RC, IFA_STRAND_BOTH = 1, 2, 3
IFA_FLAG_GRAPHS = 1
IFA_FLAG_OVERHANG = 2
IFA_FLAG_INDEXED = 4
IFA_FLAG_AUTO_MODE = 8
IFA_MAX_SEED_KS = 8

IFA_OK, IFA_E_INVALID, IFA_E_NOMEM, IFA_E_DEVICE, IFA_E_STATE, IFA_E_TOO_LONG = range(6)
STATUS = {0: "IFA_OK", 1: "IFA_E_INVALID", 2: "IFA_E_NOMEM", 3: "IFA_E_DEVICE",
          4: "IFA_E_STATE", 5: "IFA_E_TOO_LONG"}

HIT_DTYPE = np.dtype([("query", "<u4"), ("contig", "<u4"), ("pos", "<i4"), ("strand", "u1"),
                      ("n_ref", "u1"), ("mismatches", "<u2")])


class IfaConfig(ctypes.Structure):
    _fields_ = [("abi_version", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("chunk_bases", ctypes.c_uint64), ("hit_capacity", ctypes.c_uint64),
                ("strands", ctypes.c_uint32), ("n_policy", ctypes.c_uint32),
                ("sink", ctypes.c_uint32), ("host_threads", ctypes.c_uint32),
                ("work_capacity", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class IfaStats(ctypes.Structure):
    _fields_ = [("bases", ctypes.c_uint64), ("chunks", ctypes.c_uint64),
                ("kernel_launches", ctypes.c_uint64), ("rescans", ctypes.c_uint64),
                ("hits", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("pack_ms", ctypes.c_double),
                ("filter_ms", ctypes.c_double), ("filter_launches", ctypes.c_uint64),
                ("filter_windows", ctypes.c_uint64), ("work_items", ctypes.c_uint64),
                ("graph_launches", ctypes.c_uint64), ("graph_updates", ctypes.c_uint64),
                ("edge_ms", ctypes.c_double),
                ("dense_ms", ctypes.c_double), ("filter_strand_windows", ctypes.c_uint64),
                ("filter_half_strand_windows", ctypes.c_uint64),
                ("timed_passes", ctypes.c_uint64), ("timed_filter_passes", ctypes.c_uint64)]


class IfaIndexParams(ctypes.Structure):
    _fields_ = [("n_k", ctypes.c_uint32), ("k", ctypes.c_uint32 * 8), ("mask", ctypes.c_uint32),
                ("step", ctypes.c_uint32), ("prob_ppm", ctypes.c_uint32),
                ("auto_queries", ctypes.c_uint32), ("iters", ctypes.c_uint64),
                ("seed", ctypes.c_uint64)]


class IfaServerConfig(ctypes.Structure):
    _fields_ = [("max_active_queries", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("hit_budget", ctypes.c_uint64)]


class IfaServerStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_uint32), ("active", ctypes.c_uint32),
                ("active_queries", ctypes.c_uint32), ("done_waiting", ctypes.c_uint32),
                ("steps", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("step_ms", ctypes.c_double), ("cursor", ctypes.c_uint32),
                ("chunks", ctypes.c_uint32), ("hit_budget", ctypes.c_uint64),
                ("hits_reserved", ctypes.c_uint64), ("in_flight", ctypes.c_uint32),
                ("finishing", ctypes.c_uint32)]


class IfaPackedChunk(ctypes.Structure):
    _fields_ = [("n_bases", ctypes.c_uint64), ("hi", ctypes.c_void_p), ("lo", ctypes.c_void_p),
                ("n_contigs", ctypes.c_uint32), ("n_runs", ctypes.c_uint32),
                ("contig_len", ctypes.c_void_p), ("run_start", ctypes.c_void_p),
                ("run_len", ctypes.c_void_p)]


class IfaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libifa.so; raises if it was not built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise ImportError(f"{_build.LIB} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(_build.LIB)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        st = ctypes.c_int
        L.ifa_config_default.argtypes = [ctypes.POINTER(IfaConfig)]
        L.ifa_config_default.restype = None
        L.ifa_create.argtypes = [ctypes.POINTER(IfaConfig), ctypes.POINTER(vp)]
        L.ifa_create.restype = st
        L.ifa_destroy.argtypes = [vp]
        L.ifa_destroy.restype = None
        L.ifa_last_error.argtypes = [vp]
        L.ifa_last_error.restype = ctypes.c_char_p
        L.ifa_load_queries.argtypes = [vp, u32, vp, vp, vp, vp]
        L.ifa_load_queries.restype = st
        L.ifa_scan_chunk.argtypes = [vp, u32, vp, vp, ctypes.POINTER(u32)]
        L.ifa_scan_chunk.restype = st
        L.ifa_scan_packed.argtypes = [vp, ctypes.POINTER(IfaPackedChunk), ctypes.POINTER(u32)]
        L.ifa_scan_packed.restype = st
        L.ifa_collect_hits.argtypes = [vp, vp, u64, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.ifa_collect_hits.restype = st
        L.ifa_query_stats.argtypes = [vp, vp, vp]
        L.ifa_query_stats.restype = st
        L.ifa_ref_load.argtypes = [vp, u32, vp, vp, ctypes.POINTER(u32)]
        L.ifa_ref_load.restype = st
        L.ifa_scan_resident.argtypes = [vp]
        L.ifa_scan_resident.restype = st
        L.ifa_scan_resident_into.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
        L.ifa_scan_resident_into.restype = st
        L.ifa_ref_release.argtypes = [vp]
        L.ifa_ref_release.restype = st
        L.ifa_ref_info.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u32)]
        L.ifa_ref_info.restype = st
        L.ifa_get_stats.argtypes = [vp, ctypes.POINTER(IfaStats)]
        L.ifa_get_stats.restype = st
        L.ifa_reset_stats.argtypes = [vp]
        L.ifa_reset_stats.restype = st
        L.ifa_set_graphs.argtypes = [vp, ctypes.c_int]
        L.ifa_set_graphs.restype = st
        L.ifa_set_overlap.argtypes = [vp, ctypes.c_int]
        L.ifa_set_overlap.restype = st
        L.ifa_variant_count.argtypes = []
        L.ifa_variant_count.restype = u32
        L.ifa_variant_info.argtypes = [u32, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                       ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.ifa_variant_info.restype = st
        L.ifa_set_variant.argtypes = [vp, u32]
        L.ifa_set_variant.restype = st
        L.ifa_get_variant.argtypes = [vp, ctypes.POINTER(u32)]
        L.ifa_get_variant.restype = st
        L.ifa_autotune.argtypes = [vp, u64, u32, ctypes.c_char_p, ctypes.POINTER(u32), vp]
        L.ifa_autotune.restype = st
        L.ifa_query_partition.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.ifa_query_partition.restype = st
        L.ifa_device_footprint.argtypes = [vp, ctypes.POINTER(u64)]
        L.ifa_device_footprint.restype = st
        L.ifa_server_config_default.argtypes = [ctypes.POINTER(IfaServerConfig)]
        L.ifa_server_config_default.restype = None
        L.ifa_server_create.argtypes = [vp, ctypes.POINTER(IfaServerConfig), ctypes.POINTER(vp)]
        L.ifa_server_create.restype = st
        L.ifa_server_destroy.argtypes = [vp]
        L.ifa_server_destroy.restype = None
        L.ifa_server_submit.argtypes = [vp, u32, vp, vp, vp, vp, ctypes.POINTER(u64)]
        L.ifa_server_submit.restype = st
        L.ifa_server_step.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.ifa_server_step.restype = st
        L.ifa_server_poll.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.ifa_server_poll.restype = st
        L.ifa_server_take.argtypes = [vp, u64, vp, u64]
        L.ifa_server_take.restype = st
        L.ifa_server_info.argtypes = [vp, ctypes.POINTER(IfaServerStats)]
        L.ifa_server_info.restype = st
        L.ifa_index_params_default.argtypes = [ctypes.POINTER(IfaIndexParams)]
        L.ifa_index_params_default.restype = None
        L.ifa_set_index_params.argtypes = [vp, ctypes.POINTER(IfaIndexParams)]
        L.ifa_set_index_params.restype = st
        L.ifa_query_seeds.argtypes = [vp, vp, vp]
        L.ifa_query_seeds.restype = st
        L.ifa_query_mode.argtypes = [vp, ctypes.POINTER(u32)]
        L.ifa_query_mode.restype = st
        L.ifa_sam_create.argtypes = [u32, vp, vp, vp, u32, ctypes.POINTER(vp)]
        L.ifa_sam_create.restype = st
        L.ifa_sam_destroy.argtypes = [vp]
        L.ifa_sam_destroy.restype = None
        L.ifa_sam_last_error.argtypes = [vp]
        L.ifa_sam_last_error.restype = ctypes.c_char_p
        L.ifa_sam_add_contigs.argtypes = [vp, u32, u32, vp, vp]
        L.ifa_sam_add_contigs.restype = st
        L.ifa_sam_header.argtypes = [vp, vp, u64, ctypes.POINTER(u64)]
        L.ifa_sam_header.restype = st
        L.ifa_sam_format.argtypes = [vp, vp, u64, vp, u64, ctypes.POINTER(u64),
                                     ctypes.POINTER(u64)]
        L.ifa_sam_format.restype = st
        _lib = L
    return _lib


def _check(ctx, status):
    if status != 0:
        msg = lib().ifa_last_error(ctx) if ctx else b""
        raise IfaError(status, (msg or b"").decode(errors="replace"))


def _bytes(x) -> bytes:
    if isinstance(x, (bytes, bytearray)):
        return bytes(x)
    if isinstance(x, str):
        return x.encode()
    return np.ascontiguousarray(x, dtype=np.uint8).tobytes()


class _SeqArray:
    """Pointer + length arrays over a list of byte sequences (kept alive).
    A list of bytes objects of up to JOIN_BYTES in all is joined into one
    buffer and its pointers are the buffer's address plus offsets; other
    items are wrapped one by one (no copy)."""

    JOIN_BYTES = 1 << 26

    SMALL = 1024

    def __init__(self, seqs, len_dtype):
        self.keep = []
        lens = None
        if (isinstance(seqs, (list, tuple)) and 0 < len(seqs) <= self.SMALL
                and all(type(x) is bytes for x in seqs)):
            # a short list (a query set): plain ctypes arrays over the joined
            # bytes, whose buffer the pointers address directly
            joined = b"".join(seqs)
            base = ctypes.cast(ctypes.c_char_p(joined), ctypes.c_void_p).value
            ln = [len(x) for x in seqs]
            arr = (ctypes.c_void_p * len(seqs))(
                *[base + o for o in itertools.accumulate(ln[:-1], initial=0)])
            self.keep = [joined, arr]
            self.n = len(seqs)
            self.ptrs = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
            self.lens = np.array(ln, dtype=len_dtype)
            return
        if isinstance(seqs, (list, tuple)) and seqs and all(type(x) is bytes for x in seqs):
            lens = np.fromiter(map(len, seqs), dtype=np.uint64, count=len(seqs))
            if int(lens.sum()) > self.JOIN_BYTES:
                lens = None
        if lens is not None:
            buf = np.frombuffer(b"".join(seqs) or b"\0", dtype=np.uint8)
            offs = np.zeros(len(seqs), dtype=np.uint64)
            np.cumsum(lens[:-1], out=offs[1:])
            addr = np.uint64(buf.ctypes.data) + offs
            self.keep = [buf, addr]
            self.n = len(seqs)
            self.ptrs = addr.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p))
            self.lens = lens.astype(len_dtype)
            return
        ptrs, lens = [], []
        for s in seqs:
            if isinstance(s, np.ndarray):
                a = np.ascontiguousarray(s, dtype=np.uint8)
            else:
                a = np.frombuffer(_bytes(s), dtype=np.uint8)
            self.keep.append(a)
            ptrs.append(a.ctypes.data if a.size else None)
            lens.append(a.size)
        n = len(ptrs)
        self.n = n
        self.ptrs = (ctypes.c_void_p * max(n, 1))(*ptrs)
        self.lens = np.array(lens or [0], dtype=len_dtype)


def _contig_arrays(contigs):
    if hasattr(contigs, "pointer_array"):
        ptrs, lens = contigs.pointer_array()
        return ptrs, lens, contigs.n_contigs, contigs
    sa = _SeqArray(contigs, np.uint64)
    return sa.ptrs, sa.lens, sa.n, sa


# --------------------------------------------------------------------------
# the C entry points, one to one
# --------------------------------------------------------------------------

def ifa_config_default() -> IfaConfig:
    cfg = IfaConfig()
    lib().ifa_config_default(ctypes.byref(cfg))
    return cfg


def ifa_create(cfg: IfaConfig | None = None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    st = lib().ifa_create(ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(ctx))
    if st != 0:
        raise IfaError(st, "ifa_create failed")
    return ctx


def ifa_destroy(ctx):
    lib().ifa_destroy(ctx)


def ifa_last_error(ctx) -> str:
    return (lib().ifa_last_error(ctx) or b"").decode(errors="replace")


def ifa_load_queries(ctx, queries, max_subs, max_n=None):
    sa = _SeqArray(queries, np.uint32)
    ks = np.ascontiguousarray(list(max_subs) or [0], dtype=np.int32)
    mn = None if max_n is None else np.ascontiguousarray(list(max_n) or [0], dtype=np.int32)
    if len(ks) < sa.n or (mn is not None and len(mn) < sa.n):
        raise ValueError("one threshold per query is required")
    _check(ctx, lib().ifa_load_queries(ctx, sa.n, sa.ptrs, sa.lens.ctypes.data, ks.ctypes.data,
                                       None if mn is None else mn.ctypes.data))


def ifa_scan_chunk(ctx, contigs) -> int:
    ptrs, lens, n, keep = _contig_arrays(contigs)
    first = ctypes.c_uint32()
    _check(ctx, lib().ifa_scan_chunk(ctx, n, ptrs, lens.ctypes.data, ctypes.byref(first)))
    del keep
    return first.value


def ifa_scan_packed(ctx, n_bases: int, hi, lo, contig_len, run_start=None, run_len=None) -> int:
    """Scan a caller-packed chunk (see ifa_packed_chunk): hi / lo uint32
    planes, contig lengths, optional N runs. Returns the first ordinal."""
    hi = np.ascontiguousarray(hi, dtype=np.uint32)
    lo = np.ascontiguousarray(lo, dtype=np.uint32)
    cl = np.ascontiguousarray(contig_len, dtype=np.uint64)
    rs = np.ascontiguousarray(run_start if run_start is not None else [], dtype=np.uint64)
    rl = np.ascontiguousarray(run_len if run_len is not None else [], dtype=np.uint32)
    pk = IfaPackedChunk(n_bases, hi.ctypes.data, lo.ctypes.data, len(cl), len(rs),
                        cl.ctypes.data, rs.ctypes.data, rl.ctypes.data)
    first = ctypes.c_uint32()
    _check(ctx, lib().ifa_scan_packed(ctx, ctypes.byref(pk), ctypes.byref(first)))
    return first.value


def ifa_collect_hits(ctx, cap: int):
    """One call: returns (hits array of at most cap records, n_remaining)."""
    out = np.empty(max(cap, 1), dtype=HIT_DTYPE)
    nw = ctypes.c_uint64()
    nr = ctypes.c_uint64()
    _check(ctx, lib().ifa_collect_hits(ctx, out.ctypes.data, cap, ctypes.byref(nw),
                                       ctypes.byref(nr)))
    return (out if nw.value == len(out) else out[:nw.value].copy()), nr.value


def ifa_query_stats(ctx, n_queries: int):
    cnt = np.zeros(max(n_queries, 1), dtype=np.uint64)
    dig = np.zeros(max(n_queries, 1), dtype=np.uint64)
    _check(ctx, lib().ifa_query_stats(ctx, cnt.ctypes.data, dig.ctypes.data))
    return cnt[:n_queries], dig[:n_queries]


def ifa_ref_load(ctx, contigs) -> int:
    ptrs, lens, n, keep = _contig_arrays(contigs)
    first = ctypes.c_uint32()
    _check(ctx, lib().ifa_ref_load(ctx, n, ptrs, lens.ctypes.data, ctypes.byref(first)))
    del keep
    return first.value


def ifa_scan_resident(ctx):
    _check(ctx, lib().ifa_scan_resident(ctx))


def ifa_scan_resident_into(ctx, d_hits: int, cap: int) -> int:
    """Allocation-free resident scan: records go to the device buffer at
    address d_hits (cap records). Returns the hit count; raises IfaError
    (status IFA_E_NOMEM, .needed = the count) when it exceeds cap."""
    n = ctypes.c_uint64()
    status = lib().ifa_scan_resident_into(ctx, ctypes.c_void_p(d_hits), cap, ctypes.byref(n))
    if status != IFA_OK:
        err = IfaError(status, ifa_last_error(ctx))
        err.needed = n.value
        raise err
    return n.value


def ifa_ref_release(ctx):
    _check(ctx, lib().ifa_ref_release(ctx))


def ifa_ref_info(ctx):
    b = ctypes.c_uint64()
    c = ctypes.c_uint32()
    _check(ctx, lib().ifa_ref_info(ctx, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def ifa_get_stats(ctx) -> dict:
    s = IfaStats()
    _check(ctx, lib().ifa_get_stats(ctx, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in IfaStats._fields_}


def ifa_reset_stats(ctx):
    _check(ctx, lib().ifa_reset_stats(ctx))


def ifa_set_graphs(ctx, enable: bool):
    _check(ctx, lib().ifa_set_graphs(ctx, 1 if enable else 0))


def ifa_set_overlap(ctx, enable: bool):
    _check(ctx, lib().ifa_set_overlap(ctx, 1 if enable else 0))


def ifa_variant_count() -> int:
    return int(lib().ifa_variant_count())


def ifa_variant_info(v: int) -> dict:
    a, b, c, e = (ctypes.c_uint32() for _ in range(4))
    st = lib().ifa_variant_info(v, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                ctypes.byref(e))
    if st != 0:
        raise IfaError(st, f"no variant {v}")
    return {"windows_per_lane": a.value, "queries_per_iter": b.value, "workgroup": c.value,
            "encoding": e.value}


def ifa_set_variant(ctx, v: int):
    _check(ctx, lib().ifa_set_variant(ctx, v))


def ifa_get_variant(ctx) -> int:
    v = ctypes.c_uint32()
    _check(ctx, lib().ifa_get_variant(ctx, ctypes.byref(v)))
    return v.value


def ifa_autotune(ctx, calib_bases: int = 0, reps: int = 0, cache_path: str | None = None):
    """Returns (chosen variant, per-variant median ms; -1 entries = cache hit)."""
    nv = ifa_variant_count()
    ms = np.zeros(nv, dtype=np.float64)
    chosen = ctypes.c_uint32()
    _check(ctx, lib().ifa_autotune(ctx, calib_bases, reps,
                                   cache_path.encode() if cache_path else None,
                                   ctypes.byref(chosen), ms.ctypes.data))
    return chosen.value, ms


def ifa_query_partition(ctx):
    """(query strands loaded, strands taking the filter kernel)."""
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    _check(ctx, lib().ifa_query_partition(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def ifa_sparse_count(ctx) -> int:
    return ifa_query_partition(ctx)[1]


def ifa_device_footprint(ctx) -> int:
    b = ctypes.c_uint64()
    _check(ctx, lib().ifa_device_footprint(ctx, ctypes.byref(b)))
    return b.value


def ifa_server_config_default() -> IfaServerConfig:
    cfg = IfaServerConfig()
    lib().ifa_server_config_default(ctypes.byref(cfg))
    return cfg


def ifa_server_create(ctx, cfg: IfaServerConfig | None = None):
    srv = ctypes.c_void_p()
    _check(ctx, lib().ifa_server_create(ctx, ctypes.byref(cfg) if cfg is not None else None,
                                        ctypes.byref(srv)))
    return srv


def ifa_server_destroy(srv):
    lib().ifa_server_destroy(srv)


def ifa_server_submit(srv, ctx, queries, max_subs, max_n=None) -> int:
    sa = _SeqArray(queries, np.uint32)
    ks = np.ascontiguousarray(list(max_subs) or [0], dtype=np.int32)
    mn = None if max_n is None else np.ascontiguousarray(list(max_n) or [0], dtype=np.int32)
    rid = ctypes.c_uint64()
    _check(ctx, lib().ifa_server_submit(srv, sa.n, sa.ptrs, sa.lens.ctypes.data, ks.ctypes.data,
                                        None if mn is None else mn.ctypes.data,
                                        ctypes.byref(rid)))
    return rid.value


def ifa_server_step(srv, ctx):
    a, d = ctypes.c_uint32(), ctypes.c_uint32()
    _check(ctx, lib().ifa_server_step(srv, ctypes.byref(a), ctypes.byref(d)))
    return a.value, d.value


def ifa_server_poll(srv, ctx):
    rid, n = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().ifa_server_poll(srv, ctypes.byref(rid), ctypes.byref(n)))
    return rid.value, n.value


def ifa_server_take(srv, ctx, request_id: int, n_hits: int) -> np.ndarray:
    out = np.zeros(max(n_hits, 1), dtype=HIT_DTYPE)
    _check(ctx, lib().ifa_server_take(srv, request_id, out.ctypes.data, n_hits))
    return out[:n_hits]


def ifa_server_info(srv) -> dict:
    st = IfaServerStats()
    lib().ifa_server_info(srv, ctypes.byref(st))
    return {k: getattr(st, k) for k, _ in IfaServerStats._fields_}


def ifa_index_params_default() -> IfaIndexParams:
    p = IfaIndexParams()
    lib().ifa_index_params_default(ctypes.byref(p))
    return p


def ifa_set_index_params(ctx, p=None, **kw):
    """Set indexed-mode parameters: an IfaIndexParams, or keyword overrides of
    the defaults (ks=[...], mask, step, prob_ppm, iters, seed)."""
    if p is None:
        p = ifa_index_params_default()
    if "ks" in kw:
        ks = list(kw.pop("ks"))
        p.n_k = len(ks)
        for i in range(8):
            p.k[i] = ks[i] if i < len(ks) else 0
    for name, v in kw.items():
        setattr(p, name, v)
    _check(ctx, lib().ifa_set_index_params(ctx, ctypes.byref(p)))


def ifa_query_seeds(ctx, n_queries: int):
    """(k per query, thresholds [n, 2] per query and strand)."""
    k = np.zeros(max(n_queries, 1), dtype=np.uint32)
    thr = np.zeros(max(2 * n_queries, 2), dtype=np.uint32)
    _check(ctx, lib().ifa_query_seeds(ctx, k.ctypes.data, thr.ctypes.data))
    return k[:n_queries], thr[:2 * n_queries].reshape(n_queries, 2)


def ifa_query_mode(ctx) -> int:
    """1 if the loaded query set runs in indexed mode, 0 for brute force."""
    v = ctypes.c_uint32()
    _check(ctx, lib().ifa_query_mode(ctx, ctypes.byref(v)))
    return v.value


def _sam_check(w, status):
    if status != 0:
        msg = lib().ifa_sam_last_error(w) if w else b""
        raise IfaError(status, (msg or b"").decode(errors="replace"))


def _names(names):
    keep = [n.encode() if isinstance(n, str) else bytes(n) for n in names]
    return keep, (ctypes.c_char_p * max(len(keep), 1))(*keep)


def ifa_sam_create(queries, names, n_policy=IFA_N_SEPARATE):
    sa = _SeqArray(queries, np.uint32)
    keep, arr = _names(names)
    if len(keep) != sa.n:
        raise ValueError("one name per query is required")
    w = ctypes.c_void_p()
    _sam_check(None, lib().ifa_sam_create(sa.n, sa.ptrs, sa.lens.ctypes.data, arr, n_policy,
                                          ctypes.byref(w)))
    return w


def ifa_sam_destroy(w):
    lib().ifa_sam_destroy(w)


def ifa_sam_last_error(w) -> str:
    return (lib().ifa_sam_last_error(w) or b"").decode(errors="replace")


def ifa_sam_add_contigs(w, first_ordinal: int, names, lens):
    keep, arr = _names(names)
    ln = np.ascontiguousarray(list(lens) or [0], dtype=np.uint64)
    if len(ln) < len(keep):
        raise ValueError("one length per contig is required")
    _sam_check(w, lib().ifa_sam_add_contigs(w, first_ordinal, len(keep), arr, ln.ctypes.data))


def ifa_sam_header(w) -> str:
    n = ctypes.c_uint64()
    _sam_check(w, lib().ifa_sam_header(w, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(max(n.value, 1))
    _sam_check(w, lib().ifa_sam_header(w, buf, n.value, ctypes.byref(n)))
    return buf.raw[:n.value].decode()


def ifa_sam_format(w, hits, cap: int = 1 << 20, buf=None):
    """One call: returns (text, hits consumed). `buf` (a ctypes char buffer of
    at least cap bytes) may be passed in to be reused."""
    h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    if buf is None:
        buf = ctypes.create_string_buffer(max(cap, 1))
    used, nb = ctypes.c_uint64(), ctypes.c_uint64()
    _sam_check(w, lib().ifa_sam_format(w, h.ctypes.data if h.size else None, h.size, buf, cap,
                                       ctypes.byref(used), ctypes.byref(nb)))
    return ctypes.string_at(buf, nb.value).decode(), used.value


class SamWriter:
    """SAM text for the hits of one query set (convenience over ifa_sam_*)."""

    def __init__(self, queries, names, n_policy=IFA_N_SEPARATE):
        self.w = ifa_sam_create(queries, names, n_policy)
        self.n_contigs = 0
        self.buf = None

    def add_contigs(self, names, lens, first_ordinal=None):
        first = self.n_contigs if first_ordinal is None else first_ordinal
        ifa_sam_add_contigs(self.w, first, names, lens)
        self.n_contigs = first + len(names)

    def header(self) -> str:
        return ifa_sam_header(self.w)

    def format(self, hits) -> str:
        cap = 1 << 22
        if self.buf is None:
            self.buf = ctypes.create_string_buffer(cap)
        parts, i = [], 0
        while i < len(hits):
            text, used = ifa_sam_format(self.w, hits[i:], cap, self.buf)
            parts.append(text)
            i += used
        return "".join(parts)

    def close(self):
        if self.w:
            ifa_sam_destroy(self.w)
            self.w = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous-batching server over a Scanner's resident reference."""

    def __init__(self, scanner, max_active_queries=4096, hit_budget=0):
        self.scanner = scanner
        cfg = ifa_server_config_default()
        cfg.max_active_queries = max_active_queries
        cfg.hit_budget = hit_budget
        self.srv = ifa_server_create(scanner.ctx, cfg)

    def close(self):
        if self.srv:
            ifa_server_destroy(self.srv)
            self.srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, queries, max_subs, max_n=None) -> int:
        return ifa_server_submit(self.srv, self.scanner.ctx, queries, max_subs, max_n)

    def step(self):
        return ifa_server_step(self.srv, self.scanner.ctx)

    def completed(self):
        """Take every completed request: list of (request_id, hits)."""
        out = []
        while True:
            rid, n = ifa_server_poll(self.srv, self.scanner.ctx)
            if rid == 0:
                return out
            out.append((rid, ifa_server_take(self.srv, self.scanner.ctx, rid, n)))

    def info(self) -> dict:
        return ifa_server_info(self.srv)


def collect_all(ctx, batch: int = 1 << 20) -> np.ndarray:
    """Drain every held hit (two-call pattern over ifa_collect_hits: a call
    with cap 0 gives the count, then batches of at most `batch` records)."""
    _, rem = ifa_collect_hits(ctx, 0)
    parts = []
    while rem:
        h, rem = ifa_collect_hits(ctx, min(rem, batch))
        parts.append(h)
    if not parts:
        return np.zeros(0, dtype=HIT_DTYPE)
    return np.concatenate(parts) if len(parts) > 1 else parts[0]


class Scanner:
    """Owns one context; convenience over the entry points above."""

    def __init__(self, *, device=0, chunk_bases=1 << 30, hit_capacity=0,
                 strands=IFA_STRAND_BOTH, n_policy=IFA_N_SEPARATE, sink=IFA_SINK_RECORDS,
                 host_threads=0, work_capacity=0, flags=IFA_FLAG_GRAPHS):
        cfg = ifa_config_default()
        cfg.device = device
        cfg.chunk_bases = chunk_bases
        cfg.hit_capacity = hit_capacity
        cfg.strands = strands
        cfg.n_policy = n_policy
        cfg.sink = sink
        cfg.host_threads = host_threads
        cfg.work_capacity = work_capacity
        cfg.flags = flags
        self.ctx = ifa_create(cfg)
        self.n_queries = 0

    def close(self):
        if self.ctx:
            ifa_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_queries(self, queries, max_subs, max_n=None):
        ifa_load_queries(self.ctx, queries, max_subs, max_n)
        self.n_queries = len(queries)

    def scan_chunk(self, contigs) -> int:
        return ifa_scan_chunk(self.ctx, contigs)

    def scan_packed(self, n_bases, hi, lo, contig_len, run_start=None, run_len=None) -> int:
        return ifa_scan_packed(self.ctx, n_bases, hi, lo, contig_len, run_start, run_len)

    def collect(self) -> np.ndarray:
        return collect_all(self.ctx)

    def query_stats(self):
        return ifa_query_stats(self.ctx, self.n_queries)

    def ref_load(self, contigs) -> int:
        return ifa_ref_load(self.ctx, contigs)

    def scan_resident(self):
        ifa_scan_resident(self.ctx)

    def resident_bases(self) -> int:
        return ifa_ref_info(self.ctx)[0]

    def stats(self) -> dict:
        return ifa_get_stats(self.ctx)

    def scan(self, queries, contigs, max_subs, max_n=None) -> np.ndarray:
        """Load queries, stream contigs, return every hit in reference order."""
        self.load_queries(queries, max_subs, max_n)
        self.scan_chunk(contigs)
        return self.collect()
