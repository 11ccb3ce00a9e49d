"""Serving driver: replays a request trace against a resident reference.

A trace is a list of (arrival_s, queries, max_subs) in arrival order. The
driver keeps wall-clock time: a request is submitted once its arrival time
has passed, the server is stepped while it has admitted or pending work, and
a request's latency is its completion time minus its arrival time.

mode="batch": continuous batching -- every arrived request is submitted at
once and the server admits it as slots and hit budget free up; the work of
admitted requests shares each step's kernels.
mode="serial": the same kernels, one request at a time in arrival order
(first in, first out); the next request is submitted only after the previous
one completed.
"""
from __future__ import annotations

import math
import time

from . import Server


def nearest_rank(values, q):
    """q-th percentile (0..100) by nearest rank."""
    if not values:
        return float("nan")
    v = sorted(values)
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


def replay(scanner, trace, *, mode="batch", max_active_queries=4096, hit_budget=0,
           keep_hits=False, log=None):
    if mode not in ("batch", "serial"):
        raise ValueError("mode must be 'batch' or 'serial'")
    n = len(trace)
    bases = scanner.resident_bases()
    lat = [0.0] * n
    done_at = [0.0] * n
    hits = {} if keep_hits else None
    n_hits = [0] * n
    id2idx = {}
    with Server(scanner, max_active_queries=max_active_queries, hit_budget=hit_budget) as srv:
        t0 = time.perf_counter()
        i = 0
        done = 0
        in_flight = 0
        steps = 0
        while done < n:
            now = time.perf_counter() - t0
            while i < n and trace[i][0] <= now and (mode == "batch" or in_flight == 0):
                _, qs, ks = trace[i]
                id2idx[srv.submit(qs, ks)] = i
                i += 1
                in_flight += 1
            if in_flight:
                srv.step()
                steps += 1
                if log and steps % 500 == 0:
                    log(f"  {mode}: step {steps}, {done}/{n} requests done, {i} arrived "
                        f"at {time.perf_counter() - t0:.1f} s")
            elif i < n:
                time.sleep(max(0.0, trace[i][0] - (time.perf_counter() - t0)))
            for rid, h in srv.completed():
                idx = id2idx.pop(rid)
                t = time.perf_counter() - t0
                done_at[idx] = t
                lat[idx] = t - trace[idx][0]
                n_hits[idx] = len(h)
                if keep_hits:
                    hits[idx] = h
                done += 1
                in_flight -= 1
                if log and done % max(1, n // 10) == 0:
                    log(f"  {mode}: {done}/{n} requests done at {t:.1f} s")
        info = srv.info()
    makespan = max(done_at) - trace[0][0]
    total_q = sum(len(r[1]) for r in trace)
    return {
        "mode": mode,
        "requests": n,
        "queries": total_q,
        "makespan_s": makespan,
        "gbpq_per_s": total_q * bases / makespan / 1e9,
        "p50_s": nearest_rank(lat, 50),
        "p99_s": nearest_rank(lat, 99),
        "mean_s": sum(lat) / n,
        "steps": steps,
        "step_ms_total": info["step_ms"],
        "hit_budget": info["hit_budget"],
        "latencies_s": lat,
        "hits": n_hits,
        "hit_records": hits,
    }
