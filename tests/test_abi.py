"""The C ABI library: it loads, and exports every entry point include/ifa.h
declares. No compute call is made here (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ifa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ifa_[a-z_]+)\s*\(", text)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("ifa_create", "ifa_load_queries", "ifa_scan_chunk", "ifa_collect_hits",
                 "ifa_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    import paper_2607_27291_amd as ifa
    L = ifa.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", ifa._build.LIB], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (ifa_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported


def test_struct_layouts_match_header():
    import paper_2607_27291_amd as ifa
    assert ifa.HIT_DTYPE.itemsize == 16
    assert ifa.HIT_DTYPE["pos"] == np.dtype("<i4")             # signed: overhang starts < 0
    assert ctypes.sizeof(ifa.IfaConfig) == 48
    cfg = ifa.ifa_config_default()
    assert cfg.abi_version == ifa.IFA_ABI_VERSION
    assert cfg.chunk_bases == 1 << 30 and cfg.strands == 3 and cfg.sink == 0


def test_null_and_bad_arguments_are_rejected_without_a_device():
    import paper_2607_27291_amd as ifa
    L = ifa.lib()
    assert L.ifa_create(None, None) == 1                      # IFA_E_INVALID
    cfg = ifa.ifa_config_default()
    cfg.chunk_bases = 1000                                    # not a multiple of 32 / too small
    ctx = ctypes.c_void_p()
    assert L.ifa_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 1
    assert not ctx.value
    cfg = ifa.ifa_config_default()
    cfg.abi_version = 99
    assert L.ifa_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 1
    cfg = ifa.ifa_config_default()
    cfg.flags = 16                                            # no such flag
    assert L.ifa_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 1
    cfg.flags = ifa.IFA_FLAG_INDEXED | ifa.IFA_FLAG_OVERHANG  # not combined
    assert L.ifa_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 1
    cfg.flags = ifa.IFA_FLAG_AUTO_MODE | ifa.IFA_FLAG_OVERHANG
    assert L.ifa_create(ctypes.byref(cfg), ctypes.byref(ctx)) == 1
    assert (ifa.IFA_FLAG_GRAPHS, ifa.IFA_FLAG_OVERHANG, ifa.IFA_FLAG_INDEXED,
            ifa.IFA_FLAG_AUTO_MODE) == (1, 2, 4, 8)
    assert L.ifa_set_index_params(None, None) == 1
    L.ifa_destroy(None)                                       # NULL-safe
    assert L.ifa_load_queries(None, 0, None, None, None, None) == 1
    assert L.ifa_scan_chunk(None, 0, None, None, None) == 1
    assert L.ifa_collect_hits(None, None, 0, None, None) == 1


def test_binding_names_mirror_the_c_entry_points():
    import paper_2607_27291_amd as ifa
    for name in declared_functions():
        assert hasattr(ifa, name), name


def test_index_params_defaults_are_the_papers():
    """Candidate seed lengths 8, 9, 10, 12, 14; 200,000 Monte Carlo trials;
    99.9 % probability (Methods, "Algorithm Design")."""
    import paper_2607_27291_amd as ifa
    p = ifa.ifa_index_params_default()
    assert list(p.k)[:p.n_k] == [8, 9, 10, 12, 14]
    assert (p.iters, p.prob_ppm, p.mask, p.step) == (200_000, 999_000, 0, 1)
    assert p.auto_queries >= 1
    assert ctypes.sizeof(ifa.IfaIndexParams) == 72


def test_sequence_marshalling_paths_agree():
    """The binding passes a short list of bytes (a query set) through ctypes
    arrays over one joined bytes object, a longer one through one joined
    numpy buffer (pointers = its address + offsets) and any other sequence
    list item by item; all must hand the C side the same bytes and lengths,
    empty items included, and an oversized long list must fall back to the
    item-by-item path."""
    import ctypes
    import random

    import numpy as np
    import paper_2607_27291_amd as m

    rng = random.Random(17)
    seqs = [bytes(rng.choice(b"ACGTN") for _ in range(rng.choice([0, 1, 5, 31, 32, 33, 150])))
            for _ in range(m._SeqArray.SMALL + 300)]

    def contents(sa):
        ptrs = ctypes.cast(sa.ptrs, ctypes.POINTER(ctypes.c_void_p))
        return [ctypes.string_at(ptrs[i], int(sa.lens[i])) if int(sa.lens[i]) else b""
                for i in range(sa.n)]

    short = seqs[:500]
    small = m._SeqArray(short, np.uint32)
    assert type(small.keep[0]) is bytes and len(small.keep) == 2
    joined = m._SeqArray(seqs, np.uint32)
    assert isinstance(joined.keep[0], np.ndarray) and len(joined.keep) == 2
    itemwise = m._SeqArray([bytearray(s) for s in seqs], np.uint32)
    assert len(itemwise.keep) == len(seqs)
    assert joined.n == itemwise.n == len(seqs) and small.n == len(short)
    assert np.array_equal(joined.lens, itemwise.lens) and joined.lens.dtype == np.uint32
    assert np.array_equal(small.lens, itemwise.lens[:500]) and small.lens.dtype == np.uint32
    assert contents(joined) == contents(itemwise) == seqs
    assert contents(small) == short
    old = m._SeqArray.JOIN_BYTES
    try:
        m._SeqArray.JOIN_BYTES = 100       # force the fallback for the same list
        fallback = m._SeqArray(seqs, np.uint64)
    finally:
        m._SeqArray.JOIN_BYTES = old
    assert len(fallback.keep) == len(seqs) and fallback.lens.dtype == np.uint64
    assert contents(fallback) == seqs
