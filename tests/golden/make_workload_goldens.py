"""Write the full-size parity fixtures of the paper-scale and batched workloads.

Every value in the files this writes comes from the oracle (oracle/) run on
inputs from the seeded generator (synth/); nothing here runs the HIP path.
Each file holds, per query, the hit count and the wrapping 64-bit digest of
the count+digest sink (the sum over the query's hits of the SplitMix64
finaliser of the packed record), plus a fingerprint of the generated
reference so that a test on another machine can tell a generator difference
from a parity failure.

Fixtures (the oracle's cost is in parentheses, 8 host threads):
  c2_4gbp_count_digest.txt     the paper-scale workload at full size: 10
                               queries L30-36 against 4 Gbp, maxSubs 0, 4, 8
                               (about 10 minutes);
  c3_10mbp_count_digest.txt    all 10,000 batched queries (L18-50, maxSubs
                               0-16) against a 10 Mbp sample of whole contigs
                               of the 1 Gbp batched reference (about 10 min);
  c3_100q_1gbp_count_digest.txt  100 batched queries stratified over (L,
                               maxSubs), leaving out pairs expected to hit
                               more than 1e7 times, against the full 1 Gbp.

Run from the repository root:  python tests/golden/make_workload_goldens.py [c2] [c3] [c3s]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

C2_KS = (0, 4, 8)


def fingerprint(ref) -> str:
    """Contig count, total bases and a hash of the contig lengths and of
    every 4096th byte (cheap, and enough to notice a different generator)."""
    import hashlib
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(ref.lens, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(ref.buf[::4096]).tobytes())
    return f"{ref.n_contigs} {ref.total} {h.hexdigest()[:32]}"


def c3_sample_contigs(ref, target=10_000_000, seed=31):
    """Whole contigs of the 1 Gbp batched reference in a seeded random order
    until they hold at least `target` bases; returned in ordinal order."""
    rng = np.random.default_rng(seed)
    pick, acc = [], 0
    for i in rng.permutation(ref.n_contigs):
        if acc >= target:
            break
        pick.append(int(i))
        acc += int(ref.lens[i])
    return sorted(pick)


def c3_stratified_queries(queries, ks, total, n=100, max_expected=1e7):
    """n queries spread over (L // 4, maxSubs // 2) cells, in cell order,
    first query of each cell, leaving out pairs whose expected hit count on
    `total` random bases (both strands) exceeds max_expected; when there are
    fewer cells than n, the second query of each cell follows, and so on."""
    from scipy.stats import binom
    cells = {}
    for i, (q, k) in enumerate(zip(queries, ks)):
        L = len(q)
        if 2 * total * binom.cdf(k, L, 0.75) > max_expected:
            continue
        cells.setdefault((L // 4, k // 2), []).append(i)
    keys = sorted(cells)
    pick, depth = [], 0
    while len(pick) < n:
        added = False
        for key in keys:
            if depth < len(cells[key]) and len(pick) < n:
                pick.append(cells[key][depth])
                added = True
        if not added:
            break
        depth += 1
    return sorted(pick)


def write(name, header, rows):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        for line in header:
            f.write(f"# {line}\n")
        for r in rows:
            f.write(" ".join(str(x) for x in r) + "\n")
    print(f"wrote {path} ({len(rows)} rows)", flush=True)


def make_c2(threads):
    w = synth.c2_paper_scale(total=4_000_000_000)
    rows = []
    for k in C2_KS:
        t0 = time.time()
        _, cnt, dig = oracle.scan(w.queries, w.ref, [k] * len(w.queries), records=False,
                                  stats=True, threads=threads)
        print(f"c2 maxSubs {k}: {int(cnt.sum())} hits, {time.time() - t0:.0f} s", flush=True)
        rows += [(k, j, int(cnt[j]), int(dig[j])) for j in range(len(w.queries))]
    write("c2_4gbp_count_digest.txt", [
        "paper-scale workload at full size: synth.c2_paper_scale(total=4e9), 10 queries,",
        "maxSubs 0, 4, 8 (one scan each), both strands, N_SEPARATE, default maxN",
        "written by tests/golden/make_workload_goldens.py from the oracle",
        f"reference {fingerprint(w.ref)}",
        "columns: maxSubs query count digest",
    ], rows)


def make_c3(threads):
    w = synth.c3_batched(total=1_000_000_000)
    pick = c3_sample_contigs(w.ref)
    sub = w.ref.subset(pick)
    t0 = time.time()
    _, cnt, dig = oracle.scan(w.queries, sub, w.max_subs, records=False, stats=True,
                              threads=threads)
    print(f"c3 10 Mbp: {int(cnt.sum())} hits, {time.time() - t0:.0f} s", flush=True)
    write("c3_10mbp_count_digest.txt", [
        "batched workload: synth.c3_batched(total=1e9), all 10,000 queries with their maxSubs,",
        f"against whole contigs {','.join(map(str, pick))} of its reference",
        f"({sub.total} bases), scanned as ordinals 0.. in that order",
        "written by tests/golden/make_workload_goldens.py from the oracle",
        f"reference {fingerprint(w.ref)}",
        "columns: query count digest",
    ], [(j, int(cnt[j]), int(dig[j])) for j in range(len(w.queries))])


def make_c3s(threads):
    w = synth.c3_batched(total=1_000_000_000)
    pick = c3_stratified_queries(w.queries, w.max_subs, w.ref.total)
    qs = [w.queries[i] for i in pick]
    ks = [w.max_subs[i] for i in pick]
    t0 = time.time()
    _, cnt, dig = oracle.scan(qs, w.ref, ks, records=False, stats=True, threads=threads)
    print(f"c3 stratified: {int(cnt.sum())} hits, {time.time() - t0:.0f} s", flush=True)
    write("c3_100q_1gbp_count_digest.txt", [
        "batched workload: synth.c3_batched(total=1e9), 100 queries stratified over",
        "(L // 4, maxSubs // 2) with at most 1e7 expected hits each, full 1 Gbp",
        "written by tests/golden/make_workload_goldens.py from the oracle",
        f"reference {fingerprint(w.ref)}",
        "columns: batched-query-index maxSubs count digest",
    ], [(pick[j], ks[j], int(cnt[j]), int(dig[j])) for j in range(len(pick))])


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c3", "c3s"]
    threads = os.cpu_count() or 1
    for name in which:
        {"c2": make_c2, "c3": make_c3, "c3s": make_c3s}[name](threads)
