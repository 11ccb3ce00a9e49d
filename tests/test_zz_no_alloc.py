"""The allocation-free entry point (ifa_scan_resident_into) against the
ordinary resident scan (ifa_scan_resident + ifa_collect_hits), through the C
ABI: two calls in a row on one context, the second with a smaller input, and
a third call whose buffer is too small. The records are compared as sets
(the allocation-free call hands them out in no particular order) after
sorting into reference order, all six fields, bit-exact."""
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


def canonical(h):
    return np.sort(h, order=["contig", "pos", "strand", "query"])


class DeviceBuffer:
    """Device memory from the HIP runtime libifa.so itself links
    (libamdhip64.so.7, already loaded with it), so that the buffer and the
    library share one runtime whatever else the process has loaded."""

    def __init__(self, nbytes):
        import ctypes
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.ptr = ctypes.c_void_p()
        rc = self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes))
        assert rc == 0, f"hipMalloc: {rc}"

    def to_host(self, nbytes):
        import ctypes
        out = np.empty(nbytes, dtype=np.uint8)
        rc = self.hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), self.ptr,
                                ctypes.c_size_t(nbytes), 2)   # hipMemcpyDeviceToHost
        assert rc == 0, f"hipMemcpy: {rc}"
        return out

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = None


def test_scan_resident_into_equals_the_resident_scan():
    import paper_2607_27291_amd as ifa
    ifa.lib()
    rng = random.Random(7007)
    # sparse strands (long, small k) and dense ones (short, large k); N runs
    qs = [rand_dna(rng, rng.choice([20, 28, 32, 40, 64])) for _ in range(24)]
    ks = [rng.choice([0, 2, 4, 9]) if len(q) > 24 else len(q) // 2 for q in qs]
    contigs = []
    for i in range(6):
        c = bytearray(rand_dna(rng, rng.choice([3000, 40_000, 130_000]), b"ACGTACGTACGTN"))
        for _ in range(20):
            q = rng.choice(qs)
            p = rng.randrange(0, len(c) - len(q))
            c[p:p + len(q)] = q if rng.random() < 0.5 else q[::-1].translate(
                bytes.maketrans(b"ACGT", b"TGCA"))
        contigs.append(bytes(c))
    cap = 1 << 20
    buf = DeviceBuffer(cap * 16)
    with ifa.Scanner(chunk_bases=1 << 16) as s:
        s.ref_load(contigs)
        for round_, n in enumerate((len(qs), 9)):
            say(f"no-alloc round {round_}: {n} queries, {s.resident_bases()} resident bases")
            s.load_queries(qs[:n], ks[:n])
            s.scan_resident()
            want = s.collect()
            got_n = ifa.ifa_scan_resident_into(s.ctx, buf.ptr.value, cap)
            assert got_n == len(want)
            raw = buf.to_host(got_n * 16)
            got = canonical(raw.view(ifa.HIT_DTYPE).copy())
            assert np.array_equal(got, want), f"round {round_}"
        say("no-alloc: buffer too small")
        with pytest.raises(ifa.IfaError) as e:
            ifa.ifa_scan_resident_into(s.ctx, buf.ptr.value, 5)
        assert e.value.status == ifa.IFA_E_NOMEM and e.value.needed == len(want)
    buf.free()
