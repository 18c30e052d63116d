"""Pins for oracle/tabulate.py and the hierarchical table (Sec. 5, Figs. 6-7)."""
import random
from math import comb

import mpmath
import numpy as np
import pytest

from oracle import native
from oracle.tabulate import (entry_index, evaluate, n_entries, piece_ab,
                             straightforward_rows, tabulated_difference, top64)
from oracle.taylor import _forward_differences, hierarchical_table
from tests.conftest import read_golden


def _fig(name):
    out = {}
    for line in read_golden("fig6_fig7_cube.txt"):
        head, vals = line.split("|")
        fig, row = head.split()
        out[(fig, row)] = [int(v) for v in vals.split()]
    return out


def test_fig6_newton_interpolation_of_cube():
    f = _fig("x")
    vals = f[("fig6", "row0")]
    assert vals == [x ** 3 for x in range(4)]
    assert _forward_differences(vals) == f[("fig6", "coeffs")]
    # the other rows of the triangle are the differences at x = 0..
    assert _forward_differences(f[("fig6", "row1")]) == f[("fig6", "coeffs")][1:]
    assert _forward_differences(f[("fig6", "row2")]) == f[("fig6", "coeffs")][2:]


def test_fig7_tabulated_difference_of_cube():
    f = _fig("x")
    W = 128
    for l in range(4):
        row = f[("fig7", f"row{l}")]
        start = f[("fig6", "coeffs")][l:]
        assert tabulated_difference(start, len(row), W) == row


def test_cube_hierarchical_with_n1_matches_fig7():
    """With N = 1, r_j(i) = Delta^j[x^3](i): row j of Fig. 7."""
    f = _fig("x")
    T = hierarchical_table(lambda x: x ** 3, 3, 1)
    for i in range(6):
        rows = straightforward_rows(T, 3, i, 128)
        assert rows[0] == f[("fig7", "row0")][i]
        assert rows[1] == f[("fig7", "row1")][i]
        assert rows[2] == f[("fig7", "row2")][i]
        assert rows[3] == 6


@pytest.mark.parametrize("W", [128, 192, 256])
def test_hierarchical_identity_integer_polynomials(W):
    """R(i N + x) = sum_j r_j(i) C(x, j) exactly, for integer polynomials
    (the bivariate identity of Sec. 5.1); mod 2^W it holds bit for bit."""
    rng = random.Random(W)
    mask = (1 << W) - 1
    for _ in range(20):
        d = rng.randrange(1, 7)
        N = rng.choice([1, 2, 7, 64, 1 << 10])
        coef = [rng.randrange(-(1 << 70), 1 << 70) for _ in range(d + 1)]
        R = lambda x: sum(c * x ** n for n, c in enumerate(coef))
        T = [[v & mask for v in row] for row in hierarchical_table(R, d, N)]
        for _ in range(10):
            i, x = rng.randrange(0, 300), rng.randrange(0, N)
            rows = straightforward_rows(T, d, i, W)
            assert evaluate(rows, x, W) == R(i * N + x) & mask
            # rows themselves are the x-differences of R at i N
            assert rows == [v & mask for v in _forward_differences([R(i * N + m) for m in range(d + 1)])]


@pytest.mark.parametrize("W", [128, 192, 256])
def test_straightforward_equals_tabulated_difference(W):
    rng = random.Random(W + 1)
    for _ in range(15):
        d = rng.randrange(1, 8)
        T = [[rng.randrange(1 << W) for _ in range(d - j + 1)] for j in range(d + 1)]
        for j in range(d + 1):
            seq = tabulated_difference(T[j], 130, W)
            for i in range(0, 130, 7):
                assert straightforward_rows(T, d, i, W)[j] == seq[i]


def test_piece_ab_definition():
    W = 192
    half, quarter = 1 << (W - 1), 1 << (W - 2)
    rows = [half + 12345, quarter, 0]
    a, b = piece_ab(rows, W)
    assert b == 1 << 63                       # floor(2^64 * (1/2 + tiny))
    assert a == 3 << 62                       # frac(-1/4) = 3/4
    # truncation (not rounding): just below 1/2 stays below 2^63
    assert piece_ab([half - 1, 0, 0], W)[1] == (1 << 63) - 1
    assert piece_ab([0, 1, 0], W)[0] == (1 << 64) - 1   # frac(-2^-W)


def test_table_layout_helpers():
    for d in range(1, 9):
        seen = [entry_index(d, j, l) for j in range(d + 1) for l in range(d - j + 1)]
        assert seen == list(range(n_entries(d)))


@pytest.mark.parametrize("W,d", [(128, 3), (192, 3), (256, 4)])
def test_native_exhaustive_matches_python_scan(W, d):
    """The C phase-3 scan evaluates the same values as the Python
    tabulated difference; classification follows the thresholds."""
    rng = random.Random(W * d)
    L = W // 64
    n, N = 6, 3000
    rows = [[rng.randrange(1 << W) for _ in range(d + 1)] for _ in range(n)]
    limbs = np.array([[[(r >> (64 * l)) & ((1 << 64) - 1) for l in range(L)] for r in pr]
                      for pr in rows], dtype=np.uint64)
    hr_lo, hr_hi = 1 << 40, 1 << 58
    rej_lo, rej_hi = (1 << 58) + (1 << 40), (1 << 64) - (1 << 40)
    full = lambda v: np.full(n, v, np.uint64)
    counts, xs, cls = native.exhaustive_many(limbs, np.full(n, N, np.uint32), full(hr_lo),
                                             full(hr_hi), full(rej_lo), full(rej_hi), d, L)
    pos = 0
    for p in range(n):
        expect = []
        for x, v in enumerate(tabulated_difference(rows[p], N, W)):
            t = top64(v, W)
            if hr_lo <= t <= hr_hi:
                expect.append((x, 1))
            elif not (rej_lo <= t <= rej_hi):
                expect.append((x, 2))
        got = [(int(xs[pos + j]), int(cls[pos + j])) for j in range(int(counts[p]))]
        pos += int(counts[p])
        assert got == expect


# ------------------------------------------------ two levels (Sec. 5.1) ---

@pytest.mark.parametrize("Du,delta,Wu,W", [(3, 2, 192, 128), (6, 4, 320, 256), (6, 3, 320, 192)])
def test_two_level_shift_of_integer_polynomials(Du, delta, Wu, W):
    """For a polynomial V with integer coefficients (no rounding anywhere
    above the last step), the sub-interval table obtained through the
    upper table and the straightforward shift in t equals the hierarchical
    table of x -> V(t S + x) computed directly, rounded to W bits."""
    from oracle.tabulate import round_to_width, subinterval_table
    from oracle.taylor import hierarchical_table
    rng = random.Random(Du * 100 + delta)
    S, N = 1 << 20, 1 << 9
    coef = [rng.randrange(-(1 << 40), 1 << 40) for _ in range(Du + 1)]
    V = lambda x: sum(c * x ** k for k, c in enumerate(coef))
    mask = (1 << Wu) - 1
    upper = [[v & mask for v in row] for row in hierarchical_table(V, Du, S)]
    for t in (0, 1, 7, 1000, 4095):
        got = subinterval_table(upper, Du, t, N, delta, Wu, W)
        ref = hierarchical_table(lambda x: V(t * S + x), delta, N)
        assert got == [[round_to_width(v & mask, Wu, W) for v in row] for row in ref], t


def test_round_to_width_closed_forms():
    from oracle.tabulate import round_to_width
    assert round_to_width(0x17, 8, 4) == 0x1
    assert round_to_width(0x18, 8, 4) == 0x2          # tie: upwards
    assert round_to_width(0xF8, 8, 4) == 0x0          # wraps mod 2^4
    assert round_to_width(0xAB, 8, 8) == 0xAB


@pytest.mark.parametrize("fname,X0", [("exp", 1.0), ("log", 3.0), ("sin", 1.0)])
def test_two_level_table_reproduces_g(fname, X0):
    """Piece values from sub-interval tables made through the upper table
    (degree 6 over 2^36 arguments, 320-bit words) equal g(t S + i N + x)
    mod 1 to within 2^-56 at random points; the approximation, truncation
    and rounding errors of this shape are all below 2^-63."""
    from oracle.tabulate import subinterval_table
    from oracle.taylor import Job, arg_ulp, f_value, out_ulp, upper_table
    count, S, N, delta, Wu, W = 1 << 36, 1 << 24, 1 << 12, 3, 320, 192
    upper = upper_table(fname, X0, count, 20, "rn", 6, S, Wu)
    job = Job(fname, X0, count, 20, "rn", N, S // N, delta, W)
    uf = out_ulp(job)
    rng = random.Random(len(fname))
    for _ in range(10):
        t, i, x = rng.randrange(count // S), rng.randrange(S // N), rng.randrange(N)
        T = subinterval_table(upper, 6, t, N, delta, Wu, W)
        V = evaluate(straightforward_rows(T, delta, i, W), x, W)
        with mpmath.workprec(300):
            X = mpmath.mpf(X0) + (t * S + i * N + x) * arg_ulp(X0)
            g = f_value(fname, X) / uf - mpmath.mpf(1) / 2 + mpmath.mpf(2) ** -20
            diff = mpmath.mpf(V) / mpmath.mpf(2) ** W - (g - mpmath.floor(g))
            diff -= mpmath.nint(diff)
            assert abs(diff) < mpmath.mpf(2) ** -56, (t, i, x, diff)
