"""The serving loop: continuous batching must not change any request's hits.

Every request's records in the mix (admitted at different steps, sharing
kernel launches with other requests, under an admission cap) must equal its
records when served alone, and those must equal the oracle's, with tolerance
0 (integer results).
"""
import random
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_dna(rng, n):
    return bytes(rng.choice(b"ACGT") for _ in range(n))


@pytest.fixture(scope="module")
def setup():
    import paper_2607_27291_amd as ifa
    import synth
    spec = synth.c5_spec(seed=5, total=12_000_000)
    ref = synth.gen_reference(spec)
    rng = random.Random(5)
    reqs = []
    for r in range(14):
        n = max(1, int(round(np.exp(rng.uniform(0, np.log(40))))))
        qs = [rand_dna(rng, rng.randint(18, 150)) for _ in range(n)]
        ks = [rng.randint(0, len(q) // 4) for q in qs]
        reqs.append((qs, ks))
    s = ifa.Scanner(chunk_bases=1 << 21)
    s.ref_load(ref)
    yield ifa, ref, reqs, s
    s.close()


def serve_all(ifa, s, batches, max_active_queries=4096, hit_budget=0):
    """batches: list of lists of requests submitted together, one batch per
    step (later batches join a server already mid-revolution)."""
    out = {}
    with ifa.Server(s, max_active_queries=max_active_queries, hit_budget=hit_budget) as srv:
        ids = {}
        pending = list(batches)
        while pending or len(out) < sum(len(b) for b in batches):
            if pending:
                for idx, (qs, ks) in pending.pop(0):
                    ids[srv.submit(qs, ks)] = idx
            srv.step()
            for rid, h in srv.completed():
                out[ids[rid]] = h
    return out


def test_alone_equals_mix_equals_oracle(setup):
    ifa, ref, reqs, s = setup
    say("serving: alone")
    alone = {}
    for i, r in enumerate(reqs):
        alone.update(serve_all(ifa, s, [[(i, r)]]))
    say("serving: staggered mix, cap 60 queries")
    items = list(enumerate(reqs))
    batches = [items[0:3], items[3:4], [], items[4:9], items[9:14]]
    mix = serve_all(ifa, s, batches, max_active_queries=60)
    assert sorted(mix) == sorted(alone) == list(range(len(reqs)))
    total = 0
    for i in range(len(reqs)):
        assert np.array_equal(mix[i], alone[i]), i
        total += len(mix[i])
    assert total > 0
    import oracle
    for i in (0, 5, 13):
        qs, ks = reqs[i]
        want = oracle.scan(qs, ref, ks)
        assert np.array_equal(alone[i], want), i


def test_server_info_and_admission_cap(setup):
    ifa, ref, reqs, s = setup
    with ifa.Server(s, max_active_queries=1) as srv:
        for qs, ks in reqs[:3]:
            srv.submit(qs, ks)
        srv.step()
        info = srv.info()
        # one request admitted alone (a request alone is always admitted)
        assert info["active"] == 1 and info["pending"] == 2
        assert info["chunks"] == 6 and info["steps"] == 1
        done = 0
        while done < 3:
            srv.step()
            done += len(srv.completed())
        assert srv.info()["completed"] == 3


def test_small_hit_budget_defers_admission_with_identical_results(setup):
    """A hit budget below two requests' reservations (each reserves at least
    1,024 records per chunk) admits one request at a time: the others wait,
    and every request's hits equal its hits when served alone with the budget
    sized from free device memory."""
    ifa, ref, reqs, s = setup
    items = list(enumerate(reqs[:5]))
    say("serving: default budget (from free device memory)")
    free = {}
    for i, r in items:
        free.update(serve_all(ifa, s, [[(i, r)]]))
    say("serving: budget 2,000 records")
    with ifa.Server(s, hit_budget=2000) as srv:
        ids = {srv.submit(qs, ks): i for i, (qs, ks) in items}
        srv.step()
        info = srv.info()
        assert info["hit_budget"] == 2000
        assert info["active"] == 1 and info["pending"] == len(items) - 1
        out = {}
        while len(out) < len(items):
            srv.step()
            for rid, h in srv.completed():
                out[ids[rid]] = h
            assert srv.info()["active"] <= 1
    for i, _ in items:
        assert np.array_equal(out[i], free[i]), i
    with ifa.Server(s) as srv:
        assert srv.info()["hit_budget"] > 1 << 20     # sized from free device memory
