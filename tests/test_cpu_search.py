"""The multi-core SIMD CPU search (libhrcpu.so, include/hrcpu.h): its
AVX-512 form of the regular test equals the oracle's Alg. 4 instance by
instance (certification, distance value, loop passes), and its hit lists
equal brute force, on degenerate instances and on the plain search
workload's."""
import numpy as np
import pytest

import synth
from oracle.search import brute_hits_np, regular_alg4
from oracle import native


@pytest.fixture(scope="module")
def cpu():
    from paper_1211_3056_amd import _cpu
    try:
        _cpu.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return _cpu


@pytest.mark.parametrize("seed", [51, 52])
def test_filter_equals_oracle(cpu, seed):
    A, B, N, lo, D = synth.adversarial_instances(seed, 3001, max_N=1 << 20)
    ok, d, it = cpu.filter_regular(A, B, N, D, lo=lo, group=1, threads=3)
    for i in range(len(A)):
        bb = (int(B[i]) - int(lo[i])) % (1 << 64)
        r = regular_alg4(int(A[i]), bb, int(N[i]), int(D[i]))
        assert (int(ok[i]), int(d[i]), int(it[i])) == (int(r.success), r.d, r.iterations), i


def test_search_equals_bruteforce_on_degenerate_instances(cpu):
    A, B, N, lo, D = synth.adversarial_instances(53, 2500, max_N=2000)
    counts, offsets, hits = cpu.search(A, B, N, D, lo=lo, group=1, cap=1 << 10, threads=4)
    for i in range(len(A)):
        ref = brute_hits_np(int(A[i]), int(B[i]), int(N[i]), int(D[i]), lo=int(lo[i]))
        o = int(offsets[i])
        assert hits[o:o + int(counts[i])].tolist() == ref, i


def test_search_config1(cpu):
    A, B, N, D = synth.config1()
    counts, offsets, hits = cpu.search(A, B, N, D)
    rc, ro, rk = native.brute_hits_many(A, B, N, np.zeros(len(A), np.uint64),
                                        np.full(len(A), D, np.uint64))
    assert np.array_equal(counts, rc) and np.array_equal(hits, rk)
    assert cpu.simd_width() in (1, 8)


def test_search_over_many_chunks_and_threads(cpu):
    """Several work chunks (4096 instances each) on several threads: every
    instance's hits equal brute force, the CSR offsets are the running sum."""
    A, B, N, lo, D = synth.adversarial_instances(54, 3 * 4096 + 77, max_N=600)
    counts, offsets, hits = cpu.search(A, B, N, D, lo=lo, group=1, cap=1 << 12, threads=3)
    assert np.array_equal(offsets[1:], np.cumsum(counts.astype(np.uint64))[:-1])
    for i in range(0, len(A), 3):
        ref = brute_hits_np(int(A[i]), int(B[i]), int(N[i]), int(D[i]), lo=int(lo[i]))
        o = int(offsets[i])
        assert hits[o:o + int(counts[i])].tolist() == ref, i
    ok, _, _ = cpu.filter_regular(A, B, N, D, lo=lo, group=1, threads=5)
    assert not (ok.astype(bool) & (counts > 0)).any()
