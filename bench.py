#!/usr/bin/env python3
"""Benchmark: the brute-force gapless scan on one MI355X.

Default workload (the default line): the paper-scale single pass -- 10
queries of length 30-36 against a 4 Gbp synthetic reference (lognormal
contigs, median 3 Mbp; per-contig GC 35-65%; N runs covering 1e-4), one
planted copy per query per 100 Mbp, at maxSubs 0, 4 and 8. The reference is
packed and resident in device memory before timing starts. One step = three
full passes (one per maxSubs) of the 10 queries over the 4 Gbp; each pass =
the scan kernels (replayed from captured HIP graphs), the hit drain from the
device and the canonical sort of the records. Beside it, in the same JSON
line (unless --only): the kernel's roofline (dense-equivalent and issued
matrix-core fractions, HBM fraction, the op model's efficiency, measured
traffic), the oracle on this host's cores (all threads and one thread), the
same step end to end from host bytes, the batched scan (10,000 queries x 1 Gbp,
count+digest) and the serving loop (Poisson trace, batched against serial,
p50/p99, plus a run at 70% of the measured capacity).

Other workloads (--workload):
  c3  batched scan: 10,000 queries, L 18-50, maxSubs 0-16 per query, against
      1 Gbp resident, count+digest sink; one step = one pass + statistics.
  c4  streaming: 100 queries, L 20-40, maxSubs 4, against a reference
      generated on the fly by host threads, packed and streamed through the
      pinned double buffer (never resident); one step = the whole reference.
      --packed: the producer writes 2-bit planes and calls ifa_scan_packed.
  c5  serving loop: Poisson arrivals (200/s) of query sets of 1-1000
      queries (log-uniform), L 18-150, maxSubs 0-L/4, against 16 Gbp
      resident; continuous batching versus serial first-in-first-out scans
      over the same trace, plus a run at 70% of the measured capacity.
  idx indexed mode: 100,000 reads of 150 bp cut from a 4 Gbp resident
      reference with exactly s substitutions, maxSubs s, for s in 0, 4, 8,
      16 (one query set each; seed tables built on the host, seed lookup
      and verification on the GPU); reports per-level time and the recall
      of the reads' origins.
  cross brute force against indexed mode on the same resident 4 Gbp for query
      sets of 1 to 2,000 queries (L 30-36, maxSubs 4), load + scan each; the
      first count at which indexed mode is faster is the mode crossover.

Prints one JSON line. `value` is Gbp*query/s (reference bases x queries,
both strands inside one unit) over the timed steps, wall clock.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gbp·query/s scanned (exact hits) + p50/p99 serving latency on 1 MI355X"
# Peaks of MI355X.
PEAK_FP4_FLOPS = 10.1e15          # dense fp4 (e2m1) matrix cores
PEAK_HBM_BYTES = 8.0e12           # HBM3E
# 32-bit integer vector ALU: 256 CUs x 4 SIMDs x 16 lanes per clock (a wave64
# instruction issues over 4 clocks on its SIMD) x 2.4 GHz = 39.3 T lane-ops/s.
PEAK_VALU_INT32 = 256 * 4 * 16 * 2.4e9
# The method's operation model for a packed-word scan: about 10 vector ops per
# reference base x query (per 32-base word and strand: 2 XOR, 1 OR, 1 AND-NOT,
# 1 popcount; two strands), and 0.25 byte of 2-bit reference read per base
# and pass, shared by every query of the pass.
OPS_PER_BPQ = 10
BYTES_PER_BASE = 0.25
# Algorithmic VALU ops per window x query strand and 32-base word of the
# dense-strand kernels (the same five operations).
OPS_PER_WINDOW_STRAND_WORD = 5
# Matrix-core filters: flops per window x query strand of the match-count
# contraction over one 32-base prefix word (32 positions x base classes x 2:
# the dense-equivalent work), and the flops the instructions issue for it
# (the banded operand's zeros included): K steps of 64 products x 2 per output.
FLOPS_DENSE = {1: 2 * 32 * 4, 2: 2 * 32 * 3, 3: 2 * 32 * 3}
FLOPS_ISSUED = {1: 3 * 64 * 2, 2: 2 * 64 * 2, 3: 2 * 64 * 2}
# Three-class tiles that run the first K step alone (maxSubs 0 and alike)
# test the window at shift r of a group on its first 16 - r bases, 12.5 on
# average over the 8 shifts, and issue one K step.
FLOPS_DENSE_HALF = 2 * 12.5 * 3
FLOPS_ISSUED_HALF = 1 * 64 * 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "idx", "cross"])
    ap.add_argument("--counts", default="1,10,30,100,200,300,500,1000,2000",
                    help="cross: query counts at which both modes are timed")
    ap.add_argument("--subs", default="0,4,8,16",
                    help="idx: substitutions per read = maxSubs, one query set each")
    ap.add_argument("--read-len", type=int, default=150, help="idx: read length")
    ap.add_argument("--requests", type=int, default=50, help="c5: requests in the trace")
    ap.add_argument("--c5-modes", default="batch,serial,70",
                    help="c5: runs to make: batch, serial and/or 70 (batch at 70%% of capacity)")
    ap.add_argument("--requests-70", type=int, default=20,
                    help="c5: requests in the supplementary run at 70%% of capacity")
    ap.add_argument("--rate", type=float, default=200.0, help="c5: Poisson arrivals per second")
    ap.add_argument("--chunk-bases", type=int, default=None,
                    help="device chunk size in bases (c2, c3: the library default 2^30 unless "
                         "given; c5: 2^28 unless given)")
    ap.add_argument("--total", type=int, default=0, help="reference bases (0 = workload default)")
    ap.add_argument("--queries", type=int, default=0, help="query count (0 = workload default)")
    ap.add_argument("--ks", default="0,4,8", help="c2: maxSubs values, one pass each")
    ap.add_argument("--packed", action="store_true",
                    help="c4: the producer writes 2-bit planes and calls ifa_scan_packed")
    ap.add_argument("--overhang", action="store_true",
                    help="c2/c3: also report windows overhanging contig ends (soft clip)")
    ap.add_argument("--sam", action="store_true",
                    help="c2: also time the SAM text of one step's hits (host writer)")
    ap.add_argument("--median", type=float, default=0.0,
                    help="c2/c3: median contig length in bases (0 = the workload's 3 Mbp)")
    ap.add_argument("--cpu-sample", type=int, default=150_000_000,
                    help="c2: reference bases the oracle baseline scans per maxSubs on all "
                         "threads (0 = skip)")
    ap.add_argument("--cpu-sample-1t", type=int, default=8_000_000,
                    help="c2: reference bases of the one-thread oracle run")
    ap.add_argument("--only", action="store_true",
                    help="default workload: the paper-scale line alone (no end-to-end, "
                         "batched or serving sub-records)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant", type=int, default=-1,
                    help="scan kernel variant (default: autotuned on the workload's queries)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every pass eagerly (the default replays repeated resident "
                         "passes from captured HIP graphs)")
    ap.add_argument("--tune-cache", default="",
                    help="autotuner cache file (a later run with the same queries reuses "
                         "its choice)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a 1 GiB device copy kernel (calib_copy_kernel) 3 times, "
                         "to scale the HBM byte counters of a profiling run")
    return ap.parse_args()


def calib_copy():
    import ctypes
    from paper_2607_27291_amd import build as b
    L = ctypes.CDLL(b.CALIB_LIB)
    L.ifa_calib_copy.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    ms = ctypes.c_double()
    rc = L.ifa_calib_copy(1 << 30, 3, ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"calibration copy failed: HIP error {rc}")
    log(f"calib copy: 1 GiB read + 1 GiB write per launch, {ms.value:.3f} ms "
        f"({2 * (1 << 30) / ms.value / 1e6:.0f} GB/s)")


def chunk_kw(args):
    """Scanner keyword for an explicit --chunk-bases (else the library default)."""
    return {"chunk_bases": args.chunk_bases} if args.chunk_bases else {}


def choose_variant(ifa, s, args, queries, ks, calib_bases=64 << 20, reps=5):
    """Autotune the kernel variant on a calibration chunk (64 Mi random bases
    by default) with the workload's queries, unless one is given."""
    if args.variant >= 0:
        ifa.ifa_set_variant(s.ctx, args.variant)
        return None
    s.load_queries(queries, ks)
    chosen, ms = ifa.ifa_autotune(s.ctx, calib_bases, reps, args.tune_cache or None)
    log(f"autotune: variant {chosen} {ifa.ifa_variant_info(chosen)}; "
        f"ms per variant {[round(float(x), 4) for x in ms]}")
    return {"chosen": chosen, "ms": [round(float(x), 4) for x in ms]}


def choose_variant_over(ifa, s, args, queries, ks_sets):
    """Autotune over several threshold sets of the same queries (one pass each
    in a step): every variant's median times are summed over the sets and the
    fastest in total is chosen."""
    if args.variant >= 0:
        ifa.ifa_set_variant(s.ctx, args.variant)
        return None
    total = None
    for ks in ks_sets:
        s.load_queries(queries, ks)
        _, ms = ifa.ifa_autotune(s.ctx, 64 << 20, 5, None)
        ms = np.asarray(ms, dtype=np.float64)
        total = ms if total is None else total + ms
    best = int(np.argmin(total))
    ifa.ifa_set_variant(s.ctx, best)
    log(f"autotune over {len(ks_sets)} threshold sets: variant {best} "
        f"{ifa.ifa_variant_info(best)}; summed ms {[round(float(x), 4) for x in total]}")
    return {"chosen": best, "ms_summed": [round(float(x), 4) for x in total],
            "threshold_sets": len(ks_sets)}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "scan_filter_mfma3_c2_4gbp_hbm_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2607_27291_amd", "csrc", "ifa_scan.hip")


def kernel_code_sha256(path):
    """SHA-256 of a kernel source file's code: comments, trailing blanks and
    empty lines removed, so that a comment edit does not count as a change
    (any code change in the file, in any kernel, does)."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.rstrip() for ln in text.splitlines()]
    return hashlib.sha256("\n".join(ln for ln in lines if ln).encode()).hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` on the paper-scale workload from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when that
    summary is for another kernel or the kernel code changed since."""
    try:
        with open(TRAFFIC_PROFILE) as f:
            kv = dict(line.split(": ", 1) for line in f.read().splitlines() if ": " in line)
        sha = kernel_code_sha256(KERNEL_SOURCE)
    except OSError:
        return None
    if kv.get("kernel", "").strip() != kernel or kv.get("kernel_code_sha256", "").strip() != sha:
        return None
    return int(kv["traffic_bytes_per_launch"])


def op_model(gbpq_s):
    """The line's rate against the operation model's bound."""
    bound = PEAK_VALU_INT32 / OPS_PER_BPQ / 1e9
    return {"ops_per_bpq": OPS_PER_BPQ, "valu_peak_tops": round(PEAK_VALU_INT32 / 1e12, 2),
            "bound_gbpq_s": round(bound, 1), "achieved_gbpq_s": round(gbpq_s, 1),
            "efficiency": round(gbpq_s / bound, 4)}


def roofline(ifa, st, variant, traffic=False, st_k=None):
    """Roofline of the filter kernel (the dominant one), its average time per
    pass from HIP events on the stream it runs on (every filter launch of a
    pass lies between two events).
      * matrix-core filters (bound "mfma"): achieved = the dense-equivalent
        flops of the match-count contraction per window x strand
        (FLOPS_DENSE, one prefix word; FLOPS_DENSE_HALF in half-step tiles)
        x the (window start, filtered strand) pairs the passes evaluated
        (waves sent whole to the exact path are not counted) / time;
        issued_frac counts the flops the instructions issue;
      * VALU filter (bound "alu"): OPS_PER_WINDOW_STRAND_WORD ops per window
        x strand against the 32-bit vector peak;
      * hbm_frac: BYTES_PER_BASE x the bases the passes covered / time,
        against the HBM peak (the method's algorithmic reference traffic);
      * traffic: HBM bytes per pass measured by rocprofv3 (FETCH_SIZE +
        WRITE_SIZE, scaled by a copy kernel of known size) for this workload,
        while the kernel source matches the profile.
    Kernel times come from st_k (kernel_timing: eager launches) when given,
    else from st; both count only the passes whose kernels were timed."""
    passes = max(1, st["filter_launches"])
    tk = st_k if st_k is not None else st
    timed = max(1, tk["timed_filter_passes"])
    filter_s = tk["filter_ms"] * 1e-3
    ms_avg = tk["filter_ms"] / timed
    shape = ifa.ifa_variant_info(variant)
    enc = shape["encoding"]
    kernel = {0: "scan_filter_kernel", 1: "scan_filter_mfma_kernel",
              2: "scan_filter_mfma3_kernel", 3: "scan_filter_mfma3_kernel"}[enc]
    # window x strand pairs the filter evaluated, over every pass (each pass
    # with its own query set), and those of half-step tiles
    ws = tk["filter_strand_windows"]
    ws_half = tk["filter_half_strand_windows"]
    if enc in FLOPS_DENSE:
        flops = FLOPS_DENSE[enc] * (ws - ws_half) + FLOPS_DENSE_HALF * ws_half
        flops_issued = FLOPS_ISSUED[enc] * (ws - ws_half) + FLOPS_ISSUED_HALF * ws_half
        achieved = flops / filter_s / 1e12 if filter_s else 0.0
        peak = PEAK_FP4_FLOPS / 1e12
        bound, unit = "mfma", "TFLOP/s"
        issued = flops_issued / filter_s / 1e12 if filter_s else 0.0
    else:
        achieved = OPS_PER_WINDOW_STRAND_WORD * ws / filter_s / 1e12 if filter_s else 0.0
        peak = PEAK_VALU_INT32 / 1e12
        bound, unit = "alu", "TOP/s"
        issued = None
    hbm = BYTES_PER_BASE * tk["bases"] / filter_s if filter_s else 0.0
    out = {
        "bound": bound,
        "achieved": round(achieved, 3),
        "peak": round(peak, 3),
        "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": None,
        "kernel": kernel,
        "per_unit": (f"{FLOPS_DENSE[enc]} flops per window x query strand (dense-equivalent "
                     "match-count contraction over a 32-base prefix; "
                     f"{FLOPS_DENSE_HALF:g} in half-step tiles, which test 16 - shift bases)")
                    if enc in FLOPS_DENSE
                    else f"{OPS_PER_WINDOW_STRAND_WORD} ops per window x query strand",
        "half_step_share": round(ws_half / ws, 4) if ws else 0.0,
        "issued_frac": round(issued / peak, 4) if issued is not None else None,
        "hbm_achieved_gbs": round(hbm / 1e9, 1),
        "hbm_frac": round(hbm / PEAK_HBM_BYTES, 4),
        "algorithmic_bytes_per_pass": int(BYTES_PER_BASE * st["bases"] / passes),
        "variant": variant,
        "variant_shape": shape,
        "kernel_ms_avg": round(ms_avg, 4),
        "kernel_timing": ("eager launches after the timed region, one kernel at a time, "
                          "HIP events around each kernel" if st_k is not None else
                          "HIP events around each kernel of the timed region's eager passes"),
        "timed_launches": tk["timed_filter_passes"],
        "passes": st["filter_launches"],
        "windows_per_pass": st["filter_windows"] // passes,
        "work_items_per_pass": st["work_items"] // passes,
        "pass_ms_avg": round(st["kernel_ms"] / max(1, st["kernel_launches"]), 4),
    }
    if traffic:
        t = profiled_traffic(kernel)
        out["traffic"] = t
        if t:
            out["traffic_over_algorithmic"] = round(t / max(1, out["algorithmic_bytes_per_pass"]), 3)
    return out


def dense_roofline(st, dense_strands, matrix=False):
    """The dense-strand kernels: OPS_PER_WINDOW_STRAND_WORD ops per window x
    strand (one 32-base word) over their time, against the 32-bit VALU peak;
    st's timed passes only (pass kernel_timing's statistics). With `matrix`
    (a variant that counts the low-hit-rate strands of at most 32 bases on
    the matrix cores) the time covers both kinds of dense kernel, and the
    rate is the VALU operation model's equivalent."""
    ms = st["dense_ms"]
    timed = max(1, st["timed_passes"])
    bases = st["bases"] * timed / max(1, st["kernel_launches"])
    ach = OPS_PER_WINDOW_STRAND_WORD * bases * dense_strands / (ms * 1e-3) if ms else 0.0
    return {"bound": "alu", "achieved": round(ach / 1e12, 3),
            "peak": round(PEAK_VALU_INT32 / 1e12, 3), "unit": "TOP/s",
            "frac": round(ach / PEAK_VALU_INT32, 4),
            "kernel": "scan_dense_kernel + scan_dense_mfma3_kernel" if matrix else "scan_dense_kernel",
            "ms_per_pass": round(ms / timed, 3)}


def base_record(args, value, ms_per_step, config):
    return {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gbp·query/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": config,
    }


_HIP = None


def device_sync():
    """hipDeviceSynchronize: every stream of the device is idle afterwards."""
    global _HIP
    if _HIP is None:
        import ctypes
        _HIP = ctypes.CDLL("libamdhip64.so")
    rc = _HIP.hipDeviceSynchronize()
    if rc != 0:
        raise RuntimeError(f"hipDeviceSynchronize failed: {rc}")


def scanner_flags(ifa, args):
    return ((0 if args.eager else ifa.IFA_FLAG_GRAPHS) |
            (ifa.IFA_FLAG_OVERHANG if args.overhang else 0))


def add_overhang(out, args, st):
    """With --overhang: the overhanging-window kernel's share of the passes
    (st: statistics whose passes all had their kernels timed one by one)."""
    if not args.overhang:
        return
    out["config"]["workload"] += ", windows overhanging contig ends included"
    out["overhang"] = {
        "edge_ms_per_pass": round(st["edge_ms"] / max(1, st["timed_passes"]), 4),
        "share_of_kernel_time": round(st["edge_ms"] / max(st["kernel_ms"], 1e-9), 4),
    }


def time_sam(ifa, w, hit_sets):
    """SAM text of one step's hits (each maxSubs pass of the step is a
    separate query set, so a separate writer): host time and line rate."""
    names = [f"q{j}" for j in range(len(w.queries))]
    cnames = [f"chr{i}" for i in range(w.ref.n_contigs)]
    lens = [int(x) for x in w.ref.lens]
    t0 = time.perf_counter()
    lines = nbytes = 0
    for h in hit_sets:
        with ifa.SamWriter(w.queries, names) as sw:
            sw.add_contigs(cnames, lens)
            text = sw.header() + sw.format(h)
        lines += len(h)
        nbytes += len(text)
    dt = time.perf_counter() - t0
    return {"lines": lines, "bytes": nbytes, "ms": round(dt * 1e3, 3),
            "lines_per_s": round(lines / dt, 1) if dt > 0 else None}


def timed_steps(ifa, s, args, step):
    for i in range(args.warmup):
        step()
        log(f"warmup step {i} done")
    ifa.ifa_get_stats(s.ctx)
    ifa.ifa_reset_stats(s.ctx)
    device_sync()   # one GPU, so no barrier: the device is idle here
    t0 = time.perf_counter()
    res = []
    for i in range(args.steps):
        res.append(step())
        log(f"step {i} done")
    device_sync()
    elapsed = time.perf_counter() - t0
    return elapsed, ifa.ifa_get_stats(s.ctx), res


def kernel_timing(ifa, s, args, step, steps=1):
    """Statistics whose passes have their kernels timed one by one, each
    alone on the device. The timed region replays passes from captured HIP
    graphs, and a replayed pass is timed only as a whole: events recorded
    inside a graph read the kernels between them 10-15 % long. In a pass with
    both filtered and dense strands the dense kernels run beside the filter,
    so each one's own time would cover the other's work too. So the kernels'
    times per launch come from `steps` more steps launched eagerly and one
    kernel at a time (the same kernels, launch shapes and inputs), right
    after the timed region."""
    ifa.ifa_set_graphs(s.ctx, False)
    ifa.ifa_set_overlap(s.ctx, False)
    try:
        ifa.ifa_reset_stats(s.ctx)
        for _ in range(steps):
            step()
        device_sync()
        return ifa.ifa_get_stats(s.ctx)
    finally:
        ifa.ifa_set_overlap(s.ctx, True)
        ifa.ifa_set_graphs(s.ctx, not args.eager)


# --------------------------------------------------------------------------
# c2: paper-scale single pass (headline)
# --------------------------------------------------------------------------

def run_c2(args):
    import synth
    import paper_2607_27291_amd as ifa

    ks = [int(x) for x in args.ks.split(",")]
    total = args.total or 4_000_000_000
    t0 = time.time()
    w = synth.c2_paper_scale(total=total, median=args.median or 3e6)
    log(f"generated {w.ref.total / 1e9:.2f} Gbp in {w.ref.n_contigs} contigs, "
        f"{len(w.plants)} planted copies ({time.time() - t0:.1f} s)")
    nq = len(w.queries)

    s = ifa.Scanner(device=0, flags=scanner_flags(ifa, args), **chunk_kw(args))
    t0 = time.time()
    s.ref_load(w.ref)
    bases, chunks = ifa.ifa_ref_info(s.ctx)
    log(f"resident: {bases / 1e9:.2f} Gbp in {chunks} device chunks ({time.time() - t0:.1f} s)")
    tune = choose_variant_over(ifa, s, args, w.queries, [[k] * nq for k in ks])
    variant = ifa.ifa_get_variant(s.ctx)

    last_hits = []

    def step():
        found = 0
        last_hits.clear()
        for k in ks:
            s.load_queries(w.queries, [k] * nq)
            s.scan_resident()
            h = s.collect()
            last_hits.append(h)
            found += len(h)
        return found

    elapsed, st, res = timed_steps(ifa, s, args, step)
    bpq_per_step = bases * nq * len(ks)
    out = base_record(args, bpq_per_step * args.steps / elapsed / 1e9,
                      elapsed * 1e3 / args.steps, {
                          "workload": "paper-scale single pass: 10 queries L30-36 vs 4 Gbp "
                                      "resident, maxSubs 0/4/8 (one pass each per step)",
                          "reference_bases": bases,
                          "queries": nq,
                          "max_subs": ks,
                          "device_chunks": chunks,
                          "hits_per_step": sum(res) // max(1, args.steps),
                      })
    if args.median:
        out["config"]["workload"] += f", median contig {args.median:.0f} bp"
        out["config"]["contigs"] = int(w.ref.n_contigs)
    if args.sam:
        out["sam"] = time_sam(ifa, w, last_hits)
    out["kernel_only_gbpq_s"] = round(bpq_per_step * args.steps / (st["kernel_ms"] * 1e-3) / 1e9, 3)
    out["autotune"] = tune
    out["graph_launches"] = st["graph_launches"]
    # kernels timed one by one over one more step, launched eagerly
    st_k = kernel_timing(ifa, s, args, step)
    add_overhang(out, args, st_k if st_k is not None else st)
    # the committed traffic figure is for this workload at its default size
    out["roofline"] = roofline(ifa, st, variant, traffic=not args.total and not args.queries,
                               st_k=st_k)

    out["op_model"] = op_model(out["value"])
    out["op_model_kernel_only"] = op_model(out["kernel_only_gbpq_s"])
    if not args.no_cpu and args.cpu_sample > 0:
        out["cpu_baseline"] = cpu_baseline(w, ks, args.cpu_sample, args.cpu_sample_1t)
    out["_workload"] = w
    out["_variant"] = variant
    s.close()
    return out


def oracle_sample(w, bases):
    """The first contigs of the workload's reference up to `bases` bases."""
    acc, idx = 0, []
    for i in range(w.ref.n_contigs):
        if acc >= bases:
            break
        idx.append(i)
        acc += int(w.ref.lens[i])
    return idx, w.ref.subset(idx)


def cpu_baseline(w, ks, sample, sample_1t):
    """The oracle (plain C, byte compare with early exit, threads over window
    ranges) timed on this host on a bounded sample of the workload: the first
    contigs, the same queries and maxSubs values; once with the threads a
    one-GPU job gets here (all of the affinity set, at most 16) and once with
    one thread (the per-core rate)."""
    import oracle
    import synth
    nq = len(w.queries)
    affinity = len(os.sched_getaffinity(0))
    threads = synth.default_threads()
    res = {}
    for label, size, th in (("all", sample, threads), ("one", sample_1t, 1)):
        idx, sub = oracle_sample(w, size)
        t0 = time.perf_counter()
        for k in ks:
            oracle.scan(w.queries, sub, [k] * nq, threads=th)
        dt = time.perf_counter() - t0
        res[label] = (sub.total * nq * len(ks) / dt / 1e9, idx, sub.total, dt)
    v, idx, tot, dt = res["all"]
    v1, idx1, tot1, dt1 = res["one"]
    return {
        "value": round(v, 4),
        "unit": "Gbp·query/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {len(idx)} contigs ({tot / 1e6:.0f} Mbp) x {nq} queries x maxSubs "
                  f"{'/'.join(map(str, ks))}, {dt:.1f} s on {threads} threads",
        "nproc": os.cpu_count(),
        "affinity_cpus": affinity,
        "threads": threads,
        "one_thread": {"value": round(v1, 4), "unit": "Gbp·query/s",
                       "sample": f"first {len(idx1)} contigs ({tot1 / 1e6:.1f} Mbp), {dt1:.1f} s"},
    }


def c2_end_to_end(args, w, ks, variant):
    """The paper-scale step from host bytes: each maxSubs pass streams the 4
    Gbp of contigs through ifa_scan_chunk (host packing, pinned double
    buffer, copies, scan) and drains the hits; nothing is resident."""
    import synth
    import paper_2607_27291_amd as ifa
    nq = len(w.queries)
    s = ifa.Scanner(device=0, host_threads=synth.default_threads(), **chunk_kw(args))
    ifa.ifa_set_variant(s.ctx, variant)

    def step():
        n = 0
        for k in ks:
            s.load_queries(w.queries, [k] * nq)
            s.scan_chunk(w.ref)
            n += len(s.collect())
        return n

    step()
    device_sync()
    ifa.ifa_reset_stats(s.ctx)
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        hits = step()
    device_sync()
    dt = (time.perf_counter() - t0) / reps
    st = ifa.ifa_get_stats(s.ctx)
    s.close()
    bpq = w.ref.total * nq * len(ks)
    return {"gbpq_s": round(bpq / dt / 1e9, 3), "ms_per_step": round(dt * 1e3, 2),
            "hits_per_step": hits, "steps": reps,
            "pack_gbp_s": round(st["bases"] / max(st["pack_ms"] * 1e-3, 1e-9) / 1e9, 2),
            "h2d_gb_s": round(st["bases"] * BYTES_PER_BASE / max(st["h2d_ms"] * 1e-3, 1e-9) / 1e9, 2),
            "note": "host bytes in, hits out: packing and copies included"}


# --------------------------------------------------------------------------
# c3: batched scan, count+digest
# --------------------------------------------------------------------------

def run_c3(args):
    import synth
    import paper_2607_27291_amd as ifa

    total = args.total or 1_000_000_000
    nq = args.queries or 10_000
    t0 = time.time()
    w = synth.c3_batched(total=total, n_queries=nq, median=args.median or 3e6)
    log(f"generated {w.ref.total / 1e9:.2f} Gbp, {nq} queries ({time.time() - t0:.1f} s)")
    s = ifa.Scanner(device=0, sink=ifa.IFA_SINK_COUNT_DIGEST, flags=scanner_flags(ifa, args),
                    **chunk_kw(args))
    s.ref_load(w.ref)
    bases, chunks = ifa.ifa_ref_info(s.ctx)
    tune = choose_variant(ifa, s, args, w.queries, w.max_subs,
                          *((16 << 20, 3) if getattr(args, "sub", False) else (64 << 20, 5)))
    variant = ifa.ifa_get_variant(s.ctx)

    def step():
        s.load_queries(w.queries, w.max_subs)
        s.scan_resident()
        return s.query_stats()

    elapsed, st, res = timed_steps(ifa, s, args, step)
    cnt, dig = res[-1]
    bpq = bases * nq
    n_sparse = ifa.ifa_sparse_count(s.ctx)
    out = base_record(args, bpq * args.steps / elapsed / 1e9, elapsed * 1e3 / args.steps, {
        "workload": f"batched scan: {nq} queries L18-50, maxSubs 0-16, vs "
                    f"{bases / 1e9:.2f} Gbp resident, count+digest"
                    + (f", median contig {args.median:.0f} bp ({w.ref.n_contigs} contigs)"
                       if args.median else ""),
        "reference_bases": bases,
        "queries": nq,
        "device_chunks": chunks,
        "hits_per_step": int(cnt.sum()),
        "sparse_strands": n_sparse,
        "dense_strands": 2 * nq - n_sparse,
    })
    out["kernel_only_gbpq_s"] = round(bpq * args.steps / (st["kernel_ms"] * 1e-3) / 1e9, 3)
    out["pass_ms_per_step"] = round(st["kernel_ms"] / args.steps, 3)
    out["graph_launches"] = st["graph_launches"]
    out["autotune"] = tune
    out["op_model"] = op_model(out["value"])
    # kernels timed one by one over one more pass, launched eagerly
    st_k = kernel_timing(ifa, s, args, step)
    tk = st_k if st_k is not None else st
    add_overhang(out, args, tk)
    out["filter_ms_per_pass"] = round(tk["filter_ms"] / max(1, tk["timed_filter_passes"]), 3)
    out["dense_ms_per_pass"] = round(tk["dense_ms"] / max(1, tk["timed_passes"]), 3)
    out["roofline"] = roofline(ifa, st, variant, st_k=st_k)
    out["dense_roofline"] = dense_roofline(tk, 2 * nq - n_sparse,
                                           matrix=ifa.ifa_variant_info(variant)["encoding"] == 3)
    s.close()
    return out


# --------------------------------------------------------------------------
# c4: streaming from a reference generated on the fly
# --------------------------------------------------------------------------

def run_c4(args):
    import numpy as np
    import synth
    import paper_2607_27291_amd as ifa

    total = args.total or 100_000_000_000
    nq = args.queries or 100
    spec = synth.c4_spec(total=total)
    lens = synth.contig_lengths(spec)
    gcs = synth.contig_gc(spec, 0, len(lens))
    qs, ks = synth.c4_queries(n=nq)
    if args.packed:
        return run_c4_packed(args, spec, lens, gcs, qs, ks)
    batch_bases = 1 << 30
    # contig batches of about batch_bases each
    batches, cur, acc = [], [], 0
    for i, n in enumerate(lens):
        cur.append(i)
        acc += int(n)
        if acc >= batch_bases:
            batches.append(cur)
            cur, acc = [], 0
    if cur:
        batches.append(cur)
    threads = synth.default_threads()
    log(f"c4: {total / 1e9:.0f} Gbp in {len(lens)} contigs, {len(batches)} batches, {nq} queries")

    # the generator stands in for reading a reference and is the slowest
    # stage: it gets every host thread, the packer half of them
    gen_threads = threads
    s = ifa.Scanner(device=0, host_threads=max(1, threads // 2))
    tune = choose_variant(ifa, s, args, qs, ks)
    variant = ifa.ifa_get_variant(s.ctx)
    s.load_queries(qs, ks)   # the footprint below includes the query tables
    foot0 = ifa.ifa_device_footprint(s.ctx)

    # two batch buffers, written in turn: scan_chunk has packed batch b into
    # the library's pinned staging before it returns, so the producer may
    # refill b's buffer with batch b + 2 (reuse also skips first-touch faults)
    max_batch = max(int(lens[idx].sum()) for idx in batches)
    bufs = [np.empty(max_batch, dtype=np.uint8) for _ in range(2)]

    def gen_batch(b):
        idx = batches[b]
        blen = lens[idx]
        offs = np.zeros(len(idx), dtype=np.uint64)
        if len(idx) > 1:
            offs[1:] = np.cumsum(blen)[:-1]
        buf = bufs[b % 2][:int(blen.sum())]
        synth.fill_contigs(spec, idx[0], blen, gcs[idx], buf, offs, gen_threads)
        return synth.Reference(buf, offs, blen)

    gen_s = [0.0]

    def step():
        # producer thread generates batch b+1 while this thread packs and
        # streams batch b (both release the GIL inside their C code)
        s.load_queries(qs, ks)
        nxt = {}

        def produce(b):
            t = time.perf_counter()
            nxt[b] = gen_batch(b)
            gen_s[0] += time.perf_counter() - t

        th = threading.Thread(target=produce, args=(0,))
        th.start()
        for b in range(len(batches)):
            th.join()
            ref = nxt.pop(b)
            if b + 1 < len(batches):
                th = threading.Thread(target=produce, args=(b + 1,))
                th.start()
            s.scan_chunk(ref)
        return len(s.collect())

    elapsed, st, res = timed_steps(ifa, s, args, step)
    foot1 = ifa.ifa_device_footprint(s.ctx)
    bpq = total * nq
    out = base_record(args, bpq * args.steps / elapsed / 1e9, elapsed * 1e3 / args.steps, {
        "workload": f"terabase-style streaming: {nq} queries L20-40, maxSubs 4, vs "
                    f"{total / 1e9:.0f} Gbp generated on the fly, packed on host threads and "
                    "streamed through pinned double buffers",
        "reference_bases": total,
        "queries": nq,
        "contigs": len(lens),
        "hits_per_step": res[-1],
    })
    out["kernel_only_gbpq_s"] = round(bpq * args.steps / (st["kernel_ms"] * 1e-3) / 1e9, 3)
    out["gpu_busy_frac"] = round(st["kernel_ms"] / (elapsed * 1e3), 4)
    out["producer_gbp_s"] = round(total * (args.steps + args.warmup) / max(gen_s[0], 1e-9) / 1e9, 3)
    out["pack_gbp_s"] = round(st["bases"] / max(st["pack_ms"] * 1e-3, 1e-9) / 1e9, 3)
    # two bit planes per base (hi, lo) cross; N and piece ends as a sparse list
    out["h2d_gb_s"] = round(st["bases"] * BYTES_PER_BASE / max(st["h2d_ms"] * 1e-3, 1e-9) / 1e9, 3)
    out["device_footprint_bytes"] = {"before": foot0, "after": foot1}
    out["autotune"] = tune
    out["roofline"] = roofline(ifa, st, variant, st_k=kernel_timing(ifa, s, args, step))
    s.close()
    return out


def run_c4_packed(args, spec, lens, gcs, qs, ks):
    """c4 with a producer that hands over 2-bit data: each batch of whole
    contigs (at most one device chunk, 2^30 bases) is generated straight into
    the two code planes and scanned with ifa_scan_packed."""
    import synth
    import paper_2607_27291_amd as ifa
    total = int(lens.sum())
    nq = len(qs)
    cap = 1 << 30
    batches, cur, acc = [], [], 0
    for i, n in enumerate(lens):
        if acc + int(n) > cap and cur:
            batches.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += int(n)
    if cur:
        batches.append(cur)
    threads = synth.default_threads()
    log(f"c4 packed: {total / 1e9:.0f} Gbp in {len(lens)} contigs, {len(batches)} chunks, "
        f"{nq} queries")
    s = ifa.Scanner(device=0, host_threads=threads)
    tune = choose_variant(ifa, s, args, qs, ks)
    variant = ifa.ifa_get_variant(s.ctx)
    s.load_queries(qs, ks)
    foot0 = ifa.ifa_device_footprint(s.ctx)
    words = (cap + 31) // 32
    planes = [(np.empty(words, np.uint32), np.empty(words, np.uint32)) for _ in range(2)]

    def gen_batch(b):
        idx = batches[b]
        hi, lo = planes[b % 2]
        n = synth.fill_packed(spec, idx[0], lens[idx], gcs[idx], hi, lo, threads)
        return n, hi, lo, lens[idx]

    gen_s = [0.0]

    def step():
        s.load_queries(qs, ks)
        nxt = {}

        def produce(b):
            t = time.perf_counter()
            nxt[b] = gen_batch(b)
            gen_s[0] += time.perf_counter() - t

        th = threading.Thread(target=produce, args=(0,))
        th.start()
        for b in range(len(batches)):
            th.join()
            n, hi, lo, bl = nxt.pop(b)
            # ifa_scan_packed copies the planes before it returns, so the
            # producer may refill this buffer with batch b + 2
            if b + 1 < len(batches):
                th = threading.Thread(target=produce, args=(b + 1,))
                th.start()
            s.scan_packed(n, hi, lo, bl)
        return len(s.collect())

    elapsed, st, res = timed_steps(ifa, s, args, step)
    foot1 = ifa.ifa_device_footprint(s.ctx)
    bpq = total * nq
    out = base_record(args, bpq * args.steps / elapsed / 1e9, elapsed * 1e3 / args.steps, {
        "workload": f"terabase-style streaming: {nq} queries L20-40, maxSubs 4, vs "
                    f"{total / 1e9:.0f} Gbp generated on the fly straight into 2-bit planes "
                    "and streamed with ifa_scan_packed through pinned double buffers",
        "reference_bases": total,
        "queries": nq,
        "contigs": len(lens),
        "hits_per_step": res[-1],
    })
    out["kernel_only_gbpq_s"] = round(bpq * args.steps / (st["kernel_ms"] * 1e-3) / 1e9, 3)
    out["gpu_busy_frac"] = round(st["kernel_ms"] / (elapsed * 1e3), 4)
    out["producer_gbp_s"] = round(total * (args.steps + args.warmup) / max(gen_s[0], 1e-9) / 1e9, 3)
    out["h2d_gb_s"] = round(st["bases"] * BYTES_PER_BASE / max(st["h2d_ms"] * 1e-3, 1e-9) / 1e9, 3)
    out["device_footprint_bytes"] = {"before": foot0, "after": foot1}
    out["autotune"] = tune
    out["roofline"] = roofline(ifa, st, variant, st_k=kernel_timing(ifa, s, args, step))
    s.close()
    return out


# --------------------------------------------------------------------------
# c5: serving loop
# --------------------------------------------------------------------------

def run_c5(args):
    import synth
    import paper_2607_27291_amd as ifa
    from paper_2607_27291_amd import serve

    total = args.total or 16_000_000_000
    t0 = time.time()
    ref = synth.gen_reference(synth.c5_spec(total=total))
    log(f"generated {ref.total / 1e9:.1f} Gbp ({time.time() - t0:.1f} s)")
    s = ifa.Scanner(device=0, chunk_bases=args.chunk_bases or (1 << 28),
                    flags=scanner_flags(ifa, args) & ~ifa.IFA_FLAG_OVERHANG)
    s.ref_load(ref)
    bases, chunks = ifa.ifa_ref_info(s.ctx)
    del ref
    log(f"resident: {bases / 1e9:.1f} Gbp in {chunks} chunks")
    trace = synth.c5_trace(n_requests=args.requests, rate=args.rate)
    if args.variant >= 0:
        ifa.ifa_set_variant(s.ctx, args.variant)
    variant = ifa.ifa_get_variant(s.ctx)
    modes = [m for m in args.c5_modes.split(",") if m]
    res = {}
    for mode in ("batch", "serial"):
        if mode in modes:
            log(f"replaying {len(trace)} requests, {mode}")
            res[mode] = serve.replay(s, trace, mode=mode, log=log)
    rate2 = None
    if "70" in modes and "batch" in res:
        # sub-saturation run: arrivals at 70% of the capacity measured above
        mean_q = sum(len(r[1]) for r in trace) / len(trace)
        cap_req_s = res["batch"]["gbpq_per_s"] * 1e9 / (mean_q * bases)
        rate2 = 0.7 * cap_req_s
        trace2 = synth.c5_trace(n_requests=args.requests_70, rate=rate2)
        log(f"replaying {len(trace2)} requests at {rate2:.3f}/s (70% of capacity), batch")
        res["batch_70pct"] = serve.replay(s, trace2, mode="batch", log=log)
    b = res["batch"] if "batch" in res else res["serial"]
    out = base_record(args, b["gbpq_per_s"], b["makespan_s"] * 1e3, {
        "workload": f"serving loop: Poisson arrivals {args.rate:g}/s, {args.requests} requests of "
                    "1-1000 queries (log-uniform), L18-150, maxSubs 0-L/4, vs "
                    f"{bases / 1e9:.0f} Gbp resident in {chunks} chunks, continuous batching",
        "reference_bases": bases,
        "requests": args.requests,
        "queries": b["queries"],
        "variant": variant,
        "graphs": not args.eager,
    })
    out["steps"] = 1
    out["warmup"] = 0
    out["serving"] = {
        k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()
            if kk not in ("latencies_s", "hits", "hit_records")}
        for k, v in res.items()
    }
    if rate2 is not None:
        out["serving"]["batch_70pct"]["rate_per_s"] = round(rate2, 4)
    if "batch" in res and "serial" in res:
        out["serving"]["batch_over_serial"] = round(res["batch"]["gbpq_per_s"] /
                                                    res["serial"]["gbpq_per_s"], 3)
    out["serving"]["hit_budget_records"] = res[next(iter(res))].get("hit_budget")
    s.close()
    return out


# --------------------------------------------------------------------------
# idx: indexed mode, reads cut from the reference (the paper's substitution
# sweep of indexed mode: 100,000 reads of 150 bp, maxSubs 0..16, 4 Gbp)
# --------------------------------------------------------------------------

def run_idx(args):
    import synth
    import paper_2607_27291_amd as ifa

    total = args.total or 4_000_000_000
    n = args.queries or 100_000
    L = args.read_len
    levels = [int(x) for x in args.subs.split(",")]
    t0 = time.time()
    ref = synth.gen_reference(synth.c2_spec(seed=6, total=total))
    log(f"generated {ref.total / 1e9:.2f} Gbp in {ref.n_contigs} contigs ({time.time() - t0:.1f} s)")
    s = ifa.Scanner(device=0, flags=ifa.IFA_FLAG_INDEXED)
    s.ref_load(ref)
    bases, chunks = ifa.ifa_ref_info(s.ctx)
    per_level = []
    load_s = scan_s = 0.0
    for subs in levels:
        reads, origin = synth.sample_reads(ref, n, L, subs, seed=6)
        device_sync()
        t0 = time.perf_counter()
        s.load_queries(reads, [subs] * n)
        t1 = time.perf_counter()
        ifa.ifa_reset_stats(s.ctx)
        s.scan_resident()
        hits = s.collect()
        device_sync()
        t2 = time.perf_counter()
        st = ifa.ifa_get_stats(s.ctx)
        k, thr = ifa.ifa_query_seeds(s.ctx, n)
        found = set(zip(hits["query"].tolist(), hits["contig"].tolist(), hits["pos"].tolist(),
                        hits["strand"].tolist()))
        recall = sum((j, int(c), int(p), int(st_)) in found
                     for j, (c, p, st_) in enumerate(origin.tolist())) / n
        load_s += t1 - t0
        scan_s += t2 - t1
        per_level.append({"max_subs": subs, "load_s": round(t1 - t0, 3),
                          "scan_s": round(t2 - t1, 3), "kernel_ms": round(st["kernel_ms"], 2),
                          "hits": int(len(hits)), "recall": round(recall, 5),
                          "seed_k": sorted(set(int(x) for x in k)),
                          "thr_median": int(np.median(thr[:, 0]))})
        log(f"maxSubs {subs}: load {t1 - t0:.2f} s, scan {t2 - t1:.3f} s, "
            f"kernel {st['kernel_ms']:.1f} ms, {len(hits)} hits, recall {recall:.4f}")
    s.close()
    bpq = bases * n * len(levels)
    out = base_record(args, bpq / (load_s + scan_s) / 1e9, (load_s + scan_s) * 1e3 / len(levels), {
        "workload": f"indexed mode: {n} reads of {L} bp cut from {bases / 1e9:.2f} Gbp resident, "
                    f"exactly s substitutions with maxSubs s, s in {levels} (one query set each)",
        "reference_bases": bases,
        "queries": n,
        "device_chunks": chunks,
    })
    out["steps"] = len(levels)
    out["warmup"] = 0
    out["scan_only_gbpq_s"] = round(bpq / scan_s / 1e9, 3)
    out["levels"] = per_level
    return out


# --------------------------------------------------------------------------
# cross: brute force versus indexed mode by query count (the mode crossover)
# --------------------------------------------------------------------------

def run_cross(args):
    import synth
    import paper_2607_27291_amd as ifa

    total = args.total or 4_000_000_000
    counts = [int(x) for x in args.counts.split(",")]
    ref = synth.gen_reference(synth.c2_spec(seed=7, total=total))
    qs_all = synth.gen_queries(7, max(counts), 30, 36)
    ctx = {m: ifa.Scanner(device=0, flags=f) for m, f in
           (("brute", 0), ("indexed", ifa.IFA_FLAG_INDEXED))}
    for s in ctx.values():
        s.ref_load(ref)
    bases, _ = ifa.ifa_ref_info(ctx["brute"].ctx)
    rows = []
    for n in counts:
        row = {"queries": n}
        for mode, s in ctx.items():
            qs = qs_all[:n]
            for rep in range(2):          # the second run is timed (warm caches)
                device_sync()
                t0 = time.perf_counter()
                s.load_queries(qs, [4] * n)
                t1 = time.perf_counter()
                ifa.ifa_reset_stats(s.ctx)
                s.scan_resident()
                h = s.collect()
                device_sync()
                dt = time.perf_counter() - t0
            row[mode + "_s"] = round(dt, 4)
            row[mode + "_load_s"] = round(t1 - t0, 4)
            row[mode + "_kernel_ms"] = round(ifa.ifa_get_stats(s.ctx)["kernel_ms"], 3)
            row[mode + "_hits"] = int(len(h))
        rows.append(row)
        log(f"{n} queries: brute {row['brute_s']:.3f} s, indexed {row['indexed_s']:.3f} s")
    for s in ctx.values():
        s.close()
    cross = next((r["queries"] for r in rows if r["indexed_s"] < r["brute_s"]), None)
    tot_b = sum(r["brute_s"] for r in rows)
    out = base_record(args, bases * sum(counts) / tot_b / 1e9, tot_b * 1e3 / len(rows), {
        "workload": f"mode crossover: query sets of {counts} queries L30-36, maxSubs 4, vs "
                    f"{bases / 1e9:.2f} Gbp resident; brute force and indexed mode, load + scan",
        "reference_bases": bases,
    })
    out["steps"] = len(rows)
    out["warmup"] = len(rows)
    out["crossover_queries"] = cross
    out["rows"] = rows
    return out


def run_default(args):
    """The paper-scale line (the driver's), and unless --only, beside it: the
    same step end to end from host bytes, the batched scan (10,000 queries x
    1 Gbp) and the serving loop (a trace of Poisson arrivals, batched against
    serial), each measured on this GPU in the same run."""
    import copy
    out = run_c2(args)
    w, variant = out.pop("_workload"), out.pop("_variant")
    if args.only or args.total or args.queries:
        return out
    ks = [int(x) for x in args.ks.split(",")]
    log("end to end: paper-scale step from host bytes")
    out["end_to_end"] = c2_end_to_end(args, w, ks, variant)
    del w
    sub = copy.copy(args)
    sub.sub = True
    sub.steps, sub.warmup = 2, 1
    log("batched scan: 10,000 queries x 1 Gbp")
    c3 = run_c3(sub)
    out["c3"] = {k: c3[k] for k in ("value", "unit", "ms_per_step", "config", "kernel_only_gbpq_s",
                                   "filter_ms_per_pass", "dense_ms_per_pass", "pass_ms_per_step",
                                   "graph_launches", "op_model", "roofline", "dense_roofline")}
    out["c3"]["steps"], out["c3"]["warmup"] = sub.steps, sub.warmup
    log("serving loop")
    sub.requests = args.requests
    sub.requests_70 = args.requests_70
    c5 = run_c5(sub)
    out["serving"] = {"value": c5["value"], "unit": c5["unit"], "config": c5["config"],
                      **c5["serving"]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is design-only)", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        calib_copy()
    if args.workload == "c2":
        out = run_default(args)
    elif args.workload == "c3":
        out = run_c3(args)
    elif args.workload == "c4":
        out = run_c4(args)
    elif args.workload == "idx":
        out = run_idx(args)
    elif args.workload == "cross":
        out = run_cross(args)
    else:
        out = run_c5(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
