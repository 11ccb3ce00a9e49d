"""Helpers for the full-size parity fixtures under tests/golden/ (test code).

The fixtures hold the oracle's per-query hit count and digest; records from
the HIP path are reduced to the same two figures here, with the count+digest
definition of the ABI (the SplitMix64 finaliser of the packed record).
"""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def mix64(z):
    """SplitMix64 output finaliser on a uint64 array (wrapping arithmetic)."""
    z = z.astype(np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def records_digest(hits, n_queries):
    """Per-query hit count and digest of GPU records, as the count+digest
    sink defines them (the fixtures hold the oracle's)."""
    key = (hits["contig"].astype(np.uint64) << np.uint64(32)) | \
        hits["pos"].astype(np.int64).astype(np.uint64) & np.uint64(0xFFFFFFFF)
    aux = hits["strand"].astype(np.uint64) | (hits["mismatches"].astype(np.uint64) << np.uint64(1)) \
        | (hits["n_ref"].astype(np.uint64) << np.uint64(10))
    h = mix64(key ^ (aux << np.uint64(45)))
    cnt = np.bincount(hits["query"], minlength=n_queries).astype(np.uint64)
    dig = np.zeros(n_queries, dtype=np.uint64)
    np.add.at(dig, hits["query"].astype(np.int64), h)
    return cnt, dig


def load_golden(name):
    """(header lines, rows of ints) of a fixture written by
    tests/golden/make_workload_goldens.py from the oracle."""
    path = os.path.join(GOLDEN, name)
    head, rows = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                head.append(line[1:].strip())
            elif line.strip():
                rows.append([int(x) for x in line.split()])
    return head, rows


def check_fingerprint(head, ref):
    """The fixture was made from the same generated reference."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_workload_goldens", os.path.join(GOLDEN, "make_workload_goldens.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    want = next(h for h in head if h.startswith("reference "))[len("reference "):]
    assert mod.fingerprint(ref) == want, "generated reference differs from the fixture's"
    return mod
