"""Pins for oracle/search.py and the C brute force (Sec. 3.1 Eq. 1, Sec. 4)."""
import random

import numpy as np
import pytest
from hypothesis import assume, given, settings, strategies as st

from oracle import native
from oracle.cf import gap_sequence
from oracle.search import (M64, brute_hits, brute_hits_np, brute_min,
                           lefevre_alg1, regular_alg2, regular_alg4)
from tests.conftest import read_golden


# --------------------------------------------------------------- Fig. 5 ---

def _fig5():
    meta, cfgs = {}, []
    for line in read_golden("fig5_a31_b39_m45.txt"):
        if "|" in line:
            head, gaps = line.split("|")
            label, n = head.split()
            cfgs.append((label, int(n), [int(g) for g in gaps.split()]))
        else:
            k, v = line.split()
            meta[k] = int(v)
    return meta, cfgs


def _closest_left_from_gaps(gaps, b):
    pos = 0
    best = None
    for g in [0] + gaps[:-1]:
        pos += g
        if pos <= b:
            best = b - pos
    return best


def test_fig5_configurations():
    meta, cfgs = _fig5()
    for _, n, gaps in cfgs:
        assert gap_sequence(meta["a"], meta["M"], n) == gaps


def test_fig5_regular_trace_looks_ahead():
    """Alg. 2 on a = 31/45, b = 39/45: after its second iteration d is the
    distance in configuration (2, 1) of the figure (look-ahead), not (2, 0)."""
    meta, cfgs = _fig5()
    a, b, M = meta["a"], meta["b"], meta["M"]
    fig = {label: _closest_left_from_gaps(gaps, b) for label, _, gaps in cfgs}
    assert fig == {"(1,0)": 8, "(2,0)": 8, "(2,1)": 5, "(3,0)": 2}
    r = regular_alg2(a, b, 100, 0, M)
    assert r.ds[:4] == [8, 5, 2, 1]
    assert r.ds[0] == fig["(1,0)"] and r.ds[1] == fig["(2,1)"] and r.ds[2] == fig["(3,0)"]
    assert regular_alg4(a, b, 100, 0, M).ds[:4] == [8, 5, 2, 1]


# ---------------------------------------------------- brute force itself ---

def test_brute_closed_forms():
    # a = 0: every point at 0, hit iff b < D, for all k (ties ordered by k)
    assert brute_hits(0, 5, 4, 6) == [0, 1, 2, 3]
    assert brute_hits(0, 5, 4, 5) == []
    # a = 2^-64: dist(k) = b - k, hits k <= b with b - k < D, closest first
    assert brute_hits(1, 10, 100, 3) == [10, 9, 8]
    assert brute_hits(1, 1, 100, 5) == [1, 0]           # k=2.. wrap to ~2^64
    # a = 1/2: points {0, 1/2}
    assert brute_hits(1 << 63, (1 << 63) + 7, 5, 8) == [1, 3]
    # N = 0 and D = 0
    assert brute_hits(123, 456, 0, M64 - 1) == []
    assert brute_hits(123, 456, 50, 0) == []
    # window start lo shifts b
    assert brute_hits(1, 10, 100, 3, lo=4) == [6, 5, 4]


def test_brute_half_period_closed_form():
    """a = 1/2, b = 1/2 + 7/2^64: even k sit at 0 (distance 1/2 + 7), odd k at
    1/2 (distance 7).  With D = 8 every odd k hits."""
    hits = brute_hits(1 << 63, (1 << 63) + 7, 9, 8)
    assert hits == [1, 3, 5, 7]


def test_brute_count_matches_area():
    """Over many random instances the hit count is N D / 2^64 on average."""
    rng = np.random.default_rng(5)
    n, N, D = 2000, 1 << 12, 1 << 56       # expected 16 hits per instance
    A = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    B = rng.integers(0, 2 ** 64, n, dtype=np.uint64)
    counts, _, _ = native.brute_hits_many(A, B, np.full(n, N, np.uint32),
                                          np.zeros(n, np.uint64), np.full(n, D, np.uint64))
    mean = counts.mean()
    assert abs(mean - 16.0) < 0.6


@settings(max_examples=300, deadline=None)
@given(st.integers(0, M64 - 1), st.integers(0, M64 - 1), st.integers(0, 300),
       st.integers(0, M64 - 1), st.integers(0, M64 - 1))
def test_brute_python_numpy_agree(A, B, N, D, lo):
    assert brute_hits(A, B, N, D, lo=lo) == brute_hits_np(A, B, N, D, lo=lo)


def test_native_brute_matches_python():
    rng = random.Random(2)
    A, B, N, lo, D = [], [], [], [], []
    for _ in range(300):
        kind = rng.randrange(4)
        a = rng.randrange(M64)
        if kind == 1:
            a = (rng.randrange(1 << 8) << rng.randrange(40, 64)) % M64   # short period
        if kind == 2:
            a = 0
        A.append(a)
        B.append(rng.randrange(M64))
        N.append(rng.choice([0, 1, 2, 3, rng.randrange(1, 2000)]))
        lo.append(rng.randrange(M64))
        D.append(rng.choice([0, 1, M64 - 1, rng.randrange(M64), 1 << rng.randrange(50, 64)]))
    counts, offs, ks = native.brute_hits_many(np.array(A, np.uint64), np.array(B, np.uint64),
                                              np.array(N, np.uint32), np.array(lo, np.uint64),
                                              np.array(D, np.uint64))
    for i in range(len(A)):
        ref = brute_hits(A[i], B[i], N[i], D[i], lo=lo[i])
        got = ks[int(offs[i]): int(offs[i]) + int(counts[i])].tolist()
        assert got == ref, i


# -------------------------------------------- lower bounds (Alg. 1, 2, 4) ---

MODULI = [45, 97, 1 << 16, 1 << 24, M64]


@settings(max_examples=600, deadline=None)
@given(st.sampled_from(MODULI), st.data())
def test_lower_bounds_never_exceed_minimum(M, data):
    A = data.draw(st.integers(0, M - 1))
    B = data.draw(st.integers(0, M - 1))
    N = data.draw(st.integers(1, 600))
    true_min = brute_min(A, B, N, M)[0]
    for alg in (lambda: lefevre_alg1(A, B, N, 0, M),
                lambda: regular_alg2(A, B, N, 0, M),
                lambda: regular_alg4(A, B, N, 0, M),
                lambda: regular_alg2(A, B, N, 0, M, printed=True),
                lambda: regular_alg4(A, B, N, 0, M, printed=True)):
        assert alg().d <= true_min


@settings(max_examples=400, deadline=None)
@given(st.sampled_from(MODULI), st.data())
def test_alg1_is_exact_on_the_points_it_placed(M, data):
    """Alg. 1's d is the closest-left distance among the u + v points it has
    placed (Sec. 4.1: d is the distance to the closest multiple on b's left)."""
    A = data.draw(st.integers(1, M - 1))
    B = data.draw(st.integers(0, M - 1))
    N = data.draw(st.integers(2, 600))
    r = lefevre_alg1(A, B, N, 0, M)
    assume(r.u + r.v <= 20000)          # a huge last quotient places ~k N points
    assert r.d == brute_min(A, B, r.u + r.v, M)[0]


@settings(max_examples=300, deadline=None)
@given(st.sampled_from(MODULI), st.data())
def test_tests_are_sound(M, data):
    """Success (d >= D) certifies that no k < N lies in the window."""
    A = data.draw(st.integers(0, M - 1))
    B = data.draw(st.integers(0, M - 1))
    N = data.draw(st.integers(1, 400))
    D = data.draw(st.integers(0, M // 8))
    has_hit = bool(brute_hits(A, B, N, D, M))
    for r in (lefevre_alg1(A, B, N, D, M), regular_alg2(A, B, N, D, M),
              regular_alg4(A, B, N, D, M)):
        if r.success:
            assert not has_hit
    r = lefevre_alg1(A, B, N, D, M)
    if not r.success and r.u + r.v < N:      # early failure names a real hit
        assert has_hit


def test_alg2_equals_alg4():
    rng = random.Random(4)
    for _ in range(2000):
        M = rng.choice(MODULI)
        A, B, N = rng.randrange(M), rng.randrange(M), rng.randrange(1, 1 << 20)
        r2, r4 = regular_alg2(A, B, N, 0, M), regular_alg4(A, B, N, 0, M)
        assert (r2.d, r2.u, r2.v) == (r4.d, r4.u, r4.v)


def test_eq3_holds_with_swapped_updates_only():
    """Reading of Alg. 2/4's counter updates.  After each iteration the
    configuration is an (i, 0) one: u intervals of length q and v of length p
    must tile the segment (Eq. 3, scaled: v p + u q = M).  The swapped
    updates keep it at every step; the printed ones break it."""
    rng = random.Random(9)
    broken = 0
    for _ in range(500):
        A, B = rng.randrange(1, M64), rng.randrange(M64)
        r = regular_alg2(A, B, 1 << 30, 0)
        for (_, p, q, u, v) in r.trace:
            assert v * p + u * q == M64
        rp = regular_alg2(A, B, 1 << 30, 0, printed=True)
        broken += any(v * p + u * q != M64 for (_, p, q, u, v) in rp.trace)
    assert broken > 450


def test_alg1_eq2_invariant():
    """Alg. 1 keeps u p + v q = 1 (scaled: M) after every iteration."""
    rng = random.Random(12)
    for _ in range(500):
        A, B = rng.randrange(1, M64), rng.randrange(M64)
        r = lefevre_alg1(A, B, 1 << 30, 0)
        for (_, p, q, u, v) in r.trace[:-1]:
            assert u * p + v * q == M64


def test_regular_iterations_grow_like_log_n():
    """One partial quotient per iteration: on random a the number of
    iterations to reach N = 2^15 points stays within the spread that Table 4
    reports for the regular search (min 8, max 19 over exp's pieces), give
    or take the randomness of a."""
    rng = random.Random(13)
    its = [regular_alg2(rng.randrange(1, M64), rng.randrange(M64), 1 << 15, 0).iterations
           for _ in range(3000)]
    mean = sum(its) / len(its)
    assert 7.5 < mean < 12.5
    assert min(its) >= 2 and max(its) <= 40
