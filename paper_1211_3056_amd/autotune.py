"""Choice of the free parameters of an HR search job.

Rigorous choices (results never depend on them, only speed does):

* degree delta: smallest degree <= 6 whose Lagrange remainder over a whole
  sub-interval stays below eps 2^-12 (so that undecided values are rare);
* word width W: smallest of 128, 192, 256 bits whose table-rounding bound
  2^-W sum_{j+l<=delta} C(N-1, j) C(tau-1, l) stays below eps 2^-12 on every
  sub-interval;
* piece length N (when the job leaves it free): the power of two that
  minimises the modelled device time per argument, search cost
  (~ partial quotients, ~ log N, per piece of N arguments) against recheck
  cost (candidates ~ window width ~ 2 eps + truncation ~ N^2);
* work-item split ("waves per sub-interval") and tabulation depth nu (pieces
  per lane): items of similar modelled cost, 64 lanes x nu pieces each.

The model constants are calibrated from measured runs (``calibrate``) and
can be overridden; the defaults come from the MI355X measurements of the
fused pass.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import mpmath
from mpmath import mpf

from .prep import (MAX_UPPER_DEGREE, UPPER_WIDTHS, _deriv_bound, _taylor_coeffs, _ulp,
                   output_ulp_range, round_sum, upper_error)

WIDTHS = (128, 192, 256)
MARGIN_BITS = 12


@dataclass
class CostModel:
    ns_per_quotient: float = 0.0095     # device ns per partial quotient (whole GPU)
    ns_per_candidate: float = 0.035     # device ns per rechecked candidate
    ns_per_piece: float = 0.02          # tabulation, queue and bookkeeping per piece

    def piece_steps(self, N: int) -> float:
        # partial quotients to reach N points: ~ ln N / (pi^2 / (12 ln 2)) + 1
        return math.log(max(N, 2)) / 1.1866 + 1.0

    def cost(self, pieces: float, N: int, candidates: float) -> float:
        return pieces * (self.piece_steps(N) * self.ns_per_quotient + self.ns_per_piece) \
            + candidates * self.ns_per_candidate


MODEL = CostModel()


def choose_degree(fname: str, X0: float, sub_len: int, s: int, uf, max_delta: int = 6) -> int:
    with mpmath.workprec(128):
        h = _ulp(X0)
        lim = mpf(2) ** (-s - MARGIN_BITS)
        for d in range(1, max_delta + 1):
            n = d + 1
            ea = _deriv_bound(fname, mpf(X0), mpf(X0) + sub_len * h, n) * (sub_len * h) ** n \
                / (mpmath.factorial(n) * uf)
            if ea <= lim:
                return d
    raise ValueError("no degree <= %d is accurate enough; use shorter sub-intervals" % max_delta)


_DU_HINT: dict = {}


def choose_upper_degree(fname: str, X0: float, count: int, s: int, delta: int = 1) -> int:
    """A degree >= delta of a range's upper polynomial whose Lagrange
    remainder over the whole range is below eps 2^-12, with the one below it
    too large (the smallest such degree, the remainder bound falling with
    the degree on these ranges).  The last choice for the same function,
    binade, length and eps is tried first, so that a stream of similar
    jobs costs about two remainder bounds each."""
    uf = output_ulp_range(fname, X0, count)
    lim = mpf(2) ** (-s - MARGIN_BITS)
    lo = max(delta, 1)

    def ok(Du):
        return upper_error(fname, X0, count, Du, uf) <= lim

    key = (fname, math.frexp(X0)[1], count, s, lo)
    hint = _DU_HINT.get(key)
    if hint is not None and ok(hint):
        Du = hint
        while Du > lo and ok(Du - 1):
            Du -= 1
    else:
        Du = hint + 1 if hint is not None else lo
        while Du <= MAX_UPPER_DEGREE and not ok(Du):
            Du += 1
        if Du > MAX_UPPER_DEGREE:
            raise ValueError("range too wide for one upper polynomial; split it")
    _DU_HINT[key] = Du
    return Du


@functools.lru_cache(maxsize=256)
def choose_upper_width(Du: int, n_sub: int, N_max: int, tau_max: int, delta: int, s: int) -> int:
    """Narrowest upper-table width (>= 256 bits) that keeps the device's
    integer steps exact, (delta N)^Du < 2^Wu, and the share of the upper
    entries' rounding in a piece value (2^-Wu sum_m C(T-1, m), carried
    through at most 2^l C(l N, n - j) C(tau-1, l) C(N-1, j), summed over the
    kept entries) below eps 2^-24."""
    T = max(n_sub, 1)
    worst = 0
    for j in range(delta + 1):
        for l in range(delta - j + 1):
            for n in range(j + l, Du + 1):
                sm = sum(math.comb(T - 1, m) for m in range(Du - n + 1))
                worst += (sm * 2 ** l * math.comb(l * N_max, n - j)
                          * math.comb(tau_max - 1, l) * math.comb(N_max - 1, j))
    for Wu in UPPER_WIDTHS:
        if Wu < 256:
            continue
        if (delta * N_max) ** Du < 1 << Wu and worst.bit_length() + s + 24 <= Wu:
            return Wu
    raise ValueError("no upper width is wide enough")


def choose_width(shapes, delta: int, s: int) -> int:
    """shapes: iterable of (N, tau) of the job's sub-intervals."""
    worst = 0
    for N, tau in set(shapes):
        worst = max(worst, round_sum(N, tau, delta))
    need = s + MARGIN_BITS + worst.bit_length()
    for W in WIDTHS:
        if W >= need:
            return W
    raise ValueError("no supported width is wide enough")


def truncation_slope(fname: str, X0: float, uf) -> float:
    """|r_2| ~ |f''| h^2 / u_f: the truncation error is about this times C(N, 2)."""
    with mpmath.workprec(80):
        h = _ulp(X0)
        c = _taylor_coeffs(fname, mpf(X0), 2, h, uf)
        return float(abs(2 * c[2]))


def choose_N(fname: str, X0: float, count: int, s: int, uf, model: CostModel = MODEL,
             lo: int = 10, hi: int = 22) -> int:
    """Power-of-two piece length with the smallest modelled time per argument."""
    r2 = truncation_slope(fname, X0, uf)
    eps = 2.0 ** -s
    best = None
    for e in range(lo, hi + 1):
        N = 1 << e
        width = 2 * eps + r2 * N * N / 2
        t = model.cost(1.0 / N, N, width)
        if best is None or t < best[0]:
            best = (t, N)
    return best[1]


def split_sub(pieces: int, N: int, candidates: float, target_ns: float,
              model: CostModel = MODEL, max_nu: int = 64):
    """Split one sub-interval's pieces into items: list of (piece0, npieces, nu)."""
    cost = model.cost(pieces, N, candidates)
    n_items = max(1, min(pieces, int(round(cost / target_ns))))
    n_items = max(n_items, -(-pieces // (64 * max_nu)))
    per = -(-pieces // n_items)
    out = []
    p = 0
    while p < pieces:
        n = min(per, pieces - p)
        out.append((p, n, -(-n // 64)))
        p += n
    return out
