"""ifa_scan_packed (caller-packed 2-bit planes, N runs, contig table) against
ifa_scan_chunk of the same contigs as bytes and against the oracle, through
the C ABI: every record field, bit-exact, including contig ordinals across
mixed calls, N runs that start or end inside a word, lowercase and IUPAC
bytes (N runs), empty contigs, forced hit-buffer overflow and both N
policies."""
import random
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rand_dna(rng, n, alphabet=b"ACGT"):
    return bytes(rng.choice(alphabet) for _ in range(n))


def pack(contigs):
    """Test-side packing of byte contigs into the ifa_packed_chunk layout:
    hi = bit 2, lo = bit 1 of each byte; non-ACGT bytes become N runs."""
    buf = np.frombuffer(b"".join(contigs), dtype=np.uint8)
    n = len(buf)
    words = (n + 31) // 32
    bits = np.zeros(words * 32, dtype=np.uint8)

    def plane(bit):
        bits[:n] = (buf >> bit) & 1
        return np.packbits(bits.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(
            np.uint32).copy() if n else np.zeros(0, np.uint32)

    hi, lo = plane(2), plane(1)
    isn = ~np.isin(buf | 0x20, np.frombuffer(b"acgt", dtype=np.uint8))
    starts, lens = [], []
    i = 0
    idx = np.flatnonzero(isn)
    while i < len(idx):
        j = i
        while j + 1 < len(idx) and idx[j + 1] == idx[j] + 1:
            j += 1
        starts.append(int(idx[i]))
        lens.append(int(idx[j] - idx[i] + 1))
        i = j + 1
    return n, hi, lo, [len(c) for c in contigs], starts, lens


@pytest.mark.parametrize("policy", [0, 1])
def test_packed_equals_bytes_equals_oracle(policy):
    import oracle
    import paper_2607_27291_amd as ifa
    rng = random.Random(88 + policy)
    for trial in range(12):
        calls = []
        for _ in range(rng.randint(1, 4)):
            cs = []
            for _ in range(rng.randint(1, 6)):
                n = rng.choice([0, 5, 31, 32, 33, 100, 999, 5000, 20_000])
                alpha = rng.choice([b"ACGT", b"ACGTN", b"acgtNNRY", b"ACGTACGTACGTN"])
                cs.append(rand_dna(rng, n, alpha))
            calls.append(cs)
        qs = [rand_dna(rng, rng.choice([8, 16, 31, 32, 33, 40, 64, 100])) for _ in range(5)]
        ks = [rng.randint(0, len(q) // 3) for q in qs]
        chunk = rng.choice([1 << 15, 1 << 16, 1 << 20])
        hcap = rng.choice([0, 0, 64])
        allc = [c for cs in calls for c in cs]
        if sum(len(c) for cs in calls for c in cs) == 0:
            continue
        say(f"packed trial {trial} policy {policy} calls {len(calls)} chunk {chunk} hcap {hcap}")
        want = oracle.scan(qs, allc, ks, policy=policy)
        with ifa.Scanner(chunk_bases=chunk, n_policy=policy, hit_capacity=hcap) as s:
            s.load_queries(qs, ks)
            s.scan_chunk(allc)
            by_bytes = s.collect()
        with ifa.Scanner(chunk_bases=chunk, n_policy=policy, hit_capacity=hcap) as s:
            s.load_queries(qs, ks)
            ordinal = 0
            for i, cs in enumerate(calls):
                if i % 2 == 1 and rng.random() < 0.5:
                    assert s.scan_chunk(cs) == ordinal      # mixed with byte calls
                else:
                    n, hi, lo, lens, rs, rl = pack(cs)
                    assert n <= chunk
                    assert s.scan_packed(n, hi, lo, lens, rs, rl) == ordinal
                ordinal += len(cs)
            got = s.collect()
        assert np.array_equal(by_bytes, want), f"bytes, trial {trial}"
        assert np.array_equal(got, want), f"packed, trial {trial}"


def test_packed_rejects_bad_chunks():
    import paper_2607_27291_amd as ifa
    with ifa.Scanner(chunk_bases=4096) as s:
        s.load_queries([b"ACGT"], [0])
        hi = np.zeros(200, np.uint32)
        for args in ((5000, hi, hi, [5000]),                 # larger than chunk_bases
                     (100, hi, hi, [50, 40]),                # lengths do not add up
                     (100, hi, hi, [100], [10, 5], [10, 2]),  # runs not ascending
                     (100, hi, hi, [100], [95], [10])):      # run past the chunk
            with pytest.raises(ifa.IfaError) as e:
                s.scan_packed(*args)
            assert e.value.status == ifa.IFA_E_INVALID
        assert s.scan_packed(0, hi, hi, []) == 0
        assert s.scan_packed(8, hi, hi, [0, 8, 0]) == 0     # empty contigs take ordinals
        assert s.scan_chunk([b"ACGTACGT"]) == 3
