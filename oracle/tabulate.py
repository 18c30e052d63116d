"""Tabulation oracle: exact W-bit fixed point, two shift algorithms.

Sec. 5 of the paper.  A sub-interval's polynomial R_t is held as its
hierarchical table (Sec. 5.1): r_j(i) = Delta^j[R_t](i N) is a polynomial in i
of degree delta - j, stored by its forward differences in i at i = 0,

    T[j][l] = Delta_i^l r_j(0)          (j + l <= delta).

All values are fractions mod 1 held as integers mod 2^W ("W-bit words").
Because binomials C(i, l) are integers, reducing every entry mod 1 commutes
with both shift algorithms.

* ``straightforward_rows`` is the straightforward shift (Sec. 5.2): the
  upper-triangular Toeplitz matrix of binomials C(i, l) applied to the table,
  r_j(i) = sum_l T[j][l] C(i, l) mod 2^W.  It is the oracle for tabulation:
  each piece is computed on its own, sharing nothing with a sequential scan.
* ``tabulated_difference`` is the tabulated difference shift (Sec. 5.2,
  Fig. 7): Delta^{l-1}(i+1) = Delta^{l-1}(i) + Delta^l(i), additions only.
  Used here only to pin the straightforward shift (the two must agree).

Degree-1 data of piece i (the inputs of Eq. 1): b = r_0(i), a = -r_1(i), both
truncated to their top 64 bits: b = floor(2^64 frac(r_0)), a =
floor(2^64 frac(-r_1)).
"""
from __future__ import annotations

from math import comb


def n_entries(delta: int) -> int:
    """Number of table entries (j, l) with j + l <= delta."""
    return (delta + 1) * (delta + 2) // 2


def entry_index(delta: int, j: int, l: int) -> int:
    """Position of T[j][l] in the flat (j-major, then l) table order."""
    return sum(delta - jj + 1 for jj in range(j)) + l


def straightforward_rows(T, delta: int, i: int, W: int):
    """[r_0(i), ..., r_delta(i)] mod 2^W by the straightforward shift.

    T is indexable as T[j][l] (Python ints mod 2^W).
    """
    mask = (1 << W) - 1
    rows = []
    for j in range(delta + 1):
        acc = 0
        for l in range(delta - j + 1):
            acc += T[j][l] * comb(i, l)
        rows.append(acc & mask)
    return rows


def tabulated_difference(diffs, steps: int, W: int):
    """Values Delta^0(i) for i in [0, steps) by repeated additions (Fig. 7).

    ``diffs`` = [Delta^0(0), ..., Delta^g(0)] of a degree-g polynomial;
    Delta^g stays constant.
    """
    mask = (1 << W) - 1
    v = list(diffs)
    out = []
    for _ in range(steps):
        out.append(v[0])
        for l in range(len(v) - 1):
            v[l] = (v[l] + v[l + 1]) & mask
    return out


def top64(x: int, W: int) -> int:
    """floor(2^64 * (x / 2^W)) for a W-bit word x, W >= 64."""
    return x >> (W - 64)


def piece_ab(rows, W: int):
    """(a, b) of one piece: a = floor(2^64 frac(-r_1)), b = floor(2^64 frac(r_0))."""
    mask = (1 << W) - 1
    b = top64(rows[0] & mask, W)
    a = top64((-rows[1]) & mask, W)
    return a, b


def tabulate(tables, delta: int, tau: int, W: int):
    """(a, b) for every piece of every sub-interval, by straightforward shift.

    ``tables`` is a list of per-sub-interval tables T[j][l].  Returns two
    lists of length len(tables) * tau, ordered (sub-interval, piece).
    """
    a_out, b_out = [], []
    for T in tables:
        for i in range(tau):
            a, b = piece_ab(straightforward_rows(T, delta, i, W), W)
            a_out.append(a)
            b_out.append(b)
    return a_out, b_out


def evaluate(rows, k: int, W: int) -> int:
    """P_i(k) = sum_j r_j(i) C(k, j) mod 2^W: the piece polynomial of Sec. 5.1
    (R_t(k + i N) in the binomial basis) at an integer k."""
    mask = (1 << W) - 1
    acc = 0
    for j, r in enumerate(rows):
        acc += r * comb(k, j)
    return acc & mask


def round_to_width(x: int, Wu: int, W: int) -> int:
    """A Wu-bit word rounded to the nearest W-bit word (W <= Wu), mod 2^W
    (ties upwards)."""
    if Wu == W:
        return x % (1 << W)
    return ((x + (1 << (Wu - W - 1))) >> (Wu - W)) % (1 << W)


def subinterval_table(U, Du: int, t: int, N: int, delta: int, Wu: int, W: int):
    """Initial table T_t[j][l] (j + l <= delta, W-bit words) of sub-interval
    t, from the upper table U[n][m] of its range (two levels of the
    hierarchical method, Sec. 5.1):

      * straightforward shift in t (Sec. 5.2) one level up:
        D_t[n] = sum_m U[n][m] C(t, m) mod 2^Wu, the step-1 differences of
        the range's polynomial at the sub-interval's first argument;
      * R_t(x) = sum_n D_t[n] C(x, n) (Newton form);
      * the hierarchical table of R_t with steps 1 and N (Fig. 6), exact
        mod 2^Wu, keeping j + l <= delta;
      * every entry rounded once to the nearest W-bit word.
    """
    from .taylor import hierarchical_table
    D = straightforward_rows(U, Du, t, Wu)
    mask = (1 << Wu) - 1
    T = hierarchical_table(lambda x: evaluate(D, x, Wu), delta, N)
    return [[round_to_width(v & mask, Wu, W) for v in row] for row in T]
