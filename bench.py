#!/usr/bin/env python3
"""Benchmark: the brute-force gapless scan on one MI355X.

Workload (paper-scale single pass): 10 queries of length 30-36 against a
4 Gbp synthetic reference (lognormal contigs, median 3 Mbp; per-contig GC
35-65%; N runs covering 1e-4), one planted copy per query per 100 Mbp, at
maxSubs 0, 4 and 8. The reference is packed and resident in device memory
before timing starts. One step = three full passes (one per maxSubs) of the
10 queries over the 4 Gbp, each pass = the scan kernels, the hit drain from
the device and the canonical sort of the records.

Prints one JSON line. `value` is Gbp*query/s (reference bases x queries,
both strands inside one unit) over the timed steps, wall clock.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gbp·query/s scanned (exact hits) + p50/p99 serving latency on 1 MI355X"
PEAK_VALU_OPS = 256 * 64 * 2.4e9        # int32 VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
# Algorithmic VALU ops per window x strand x query for the packed-word filter
# on gfx950: two v_bitop3_b32 (the mismatch bits of 32 bases), one
# v_bcnt_u32_b32 and half a v_min3_u32 (threshold fold over the windows).
OPS_PER_WINDOW_STRAND = 3.5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--total", type=int, default=4_000_000_000, help="reference bases")
    ap.add_argument("--ks", default="0,4,8")
    ap.add_argument("--cpu-sample", type=int, default=250_000_000,
                    help="reference bases the oracle baseline scans per maxSubs (0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant", type=int, default=-1,
                    help="scan kernel variant (default: autotuned on the workload's queries)")
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is design-only)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import synth
    import paper_2607_27291_amd as ifa

    if args.calib_copy:
        calib_copy()
    ks = [int(x) for x in args.ks.split(",")]
    t0 = time.time()
    w = synth.c2_paper_scale(total=args.total)
    log(f"generated {w.ref.total / 1e9:.2f} Gbp in {w.ref.n_contigs} contigs, "
        f"{len(w.plants)} planted copies ({time.time() - t0:.1f} s)")
    nq = len(w.queries)

    s = ifa.Scanner(device=0)
    t0 = time.time()
    s.ref_load(w.ref)
    bases, chunks = ifa.ifa_ref_info(s.ctx)
    log(f"resident: {bases / 1e9:.2f} Gbp in {chunks} device chunks ({time.time() - t0:.1f} s)")

    # choose the kernel variant: autotuner on a 64 Mi-base calibration chunk
    # with this workload's queries (maxSubs 4), unless one is given
    if args.variant >= 0:
        ifa.ifa_set_variant(s.ctx, args.variant)
        tune = None
    else:
        s.load_queries(w.queries, [4] * nq)
        chosen, ms = ifa.ifa_autotune(s.ctx, 64 << 20, 5)
        tune = {"chosen": chosen, "ms": [round(float(x), 4) for x in ms]}
        log(f"autotune: variant {chosen} {ifa.ifa_variant_info(chosen)}; "
            f"ms per variant {tune['ms']}")
    variant = ifa.ifa_get_variant(s.ctx)

    def step():
        found = 0
        for k in ks:
            s.load_queries(w.queries, [k] * nq)
            s.scan_resident()
            found += len(s.collect())
        return found

    for i in range(args.warmup):
        step()
        log(f"warmup step {i} done")
    ifa.ifa_get_stats(s.ctx)
    ifa.ifa_reset_stats(s.ctx)
    t0 = time.perf_counter()
    hits = 0
    for i in range(args.steps):
        hits += step()
        log(f"step {i} done")
    elapsed = time.perf_counter() - t0
    st = ifa.ifa_get_stats(s.ctx)

    bpq_per_step = bases * nq * len(ks)
    value = bpq_per_step * args.steps / elapsed / 1e9
    ms_per_step = elapsed * 1e3 / args.steps
    # dominant kernel: the filter (hot loop), timed alone by HIP events on the
    # compute stream around each of its launches
    launches = max(1, st["filter_launches"])
    filter_ms_avg = st["filter_ms"] / launches
    # algorithmic VALU ops of one launch: every window of a chunk x 2 strands x queries
    ops_per_launch = OPS_PER_WINDOW_STRAND * 2 * nq * (bases / chunks)
    achieved = ops_per_launch / (filter_ms_avg * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12
    kernel_rate = bpq_per_step * args.steps / (st["kernel_ms"] * 1e-3) / 1e9

    out = {
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
        "config": {
            "workload": "paper-scale single pass: 10 queries L30-36 vs 4 Gbp resident, "
                        "maxSubs 0/4/8 (one pass each per step)",
            "reference_bases": bases,
            "queries": nq,
            "max_subs": ks,
            "device_chunks": chunks,
            "hits_per_step": hits // max(1, args.steps),
        },
        "kernel_only_gbpq_s": round(kernel_rate, 3),
        "autotune": tune,
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(peak, 3),
            "unit": "TOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": None,
            "kernel": "scan_filter_kernel",
            "variant": variant,
            "variant_shape": ifa.ifa_variant_info(variant),
            "kernel_ms_avg": round(filter_ms_avg, 4),
            "launches": launches,
            "pass_ms_avg": round(st["kernel_ms"] / max(1, st["kernel_launches"]), 4),
        },
    }

    if not args.no_cpu and args.cpu_sample > 0:
        import oracle
        # bounded sample: the first contigs up to cpu_sample bases
        acc, idx = 0, []
        for i in range(w.ref.n_contigs):
            if acc >= args.cpu_sample:
                break
            idx.append(i)
            acc += int(w.ref.lens[i])
        sub = w.ref.subset(idx)
        threads = synth.default_threads()
        t0 = time.perf_counter()
        for k in ks:
            oracle.scan(w.queries, sub, [k] * nq, threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(sub.total * nq * len(ks) / dt / 1e9, 4),
            "unit": "Gbp·query/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"first {len(idx)} contigs ({sub.total / 1e6:.0f} Mbp) x 10 queries x "
                      f"maxSubs {'/'.join(map(str, ks))}, {dt:.1f} s",
        }
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
