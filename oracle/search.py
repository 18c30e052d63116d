"""Degree-1 search (oracle): brute force and the paper's lower-bound tests.

The degree-1 question of the paper (Sec. 3.1, Eq. 1): given a, b in [0, 1)
and N, is min{ (b - a x) mod 1 | x < N } below the threshold?  The search on
the hot path returns the whole set behind that minimum:

    H(A, B, N, lo, D) = { k in [0, N) : (B - lo - k A) mod M < D }

with a = A/M, b = B/M (M = 2^64 on the hot path), a window start lo and a
width D (hit iff strictly below D).  ``brute_hits`` is that definition
written out; it is the oracle for the search.  Hits are listed by increasing
distance (B - lo - k A) mod M, ties (coincident points) by increasing k; the
distance order is unique because distinct points have distinct distances.

``lefevre_alg1``, ``regular_alg2`` and ``regular_alg4`` follow Alg. 1, 2 and 4
of Sec. 4 over a generic modulus M.  They compute a lower bound d on the
minimum (they place n >= N points, Sec. 4.1).  Readings taken where the
printed algorithms are ambiguous:

* the threshold input is the full one-sided window D = 2 eps'' of Eq. 1, and a
  test certifies "no hit" iff d >= D (strict-below hit rule);
* Alg. 2/4 as printed update u and v the wrong way round for their own text
  (u, v hold q_i, q_{i-1} for even i) and for Eq. 3; the default here swaps the
  two updates (v += k u when q is reduced, u += k v when p is reduced).
  ``printed=True`` runs the printed form; both give valid lower bounds, only
  the exit count differs;
* Alg. 4's "d = d - p mod q" is read as (d - p) mod q, as in Alg. 2;
* a zero remainder (A/M rational, the point set has become periodic) ends the
  loop: every distinct point has been placed and d is exact.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

M64 = 1 << 64


def brute_hits(A: int, B: int, N: int, D: int, M: int = M64, lo: int = 0):
    """Sorted hit list of one instance by exhaustive evaluation (Eq. 1).

    Returns the list of k in [0, N) with (B - lo - k A) mod M < D, ordered by
    (distance, k).  Pure Python integers: exact for any modulus.
    """
    hits = []
    for k in range(N):
        dist = (B - lo - k * A) % M
        if dist < D:
            hits.append((dist, k))
    hits.sort()
    return [k for _, k in hits]


def brute_hits_np(A: int, B: int, N: int, D: int, lo: int = 0):
    """Same as ``brute_hits`` for M = 2^64, vectorised with numpy uint64.

    numpy uint64 array arithmetic wraps modulo 2^64, which is exactly the
    fixed-point arithmetic mod 1 of the definition.
    """
    if N == 0:
        return []
    k = np.arange(N, dtype=np.uint64)
    with np.errstate(over="ignore"):
        dist = np.uint64((B - lo) % M64) - k * np.uint64(A % M64)
    mask = dist < np.uint64(D) if D < M64 else np.ones(N, bool)
    ks = k[mask]
    ds = dist[mask]
    order = np.lexsort((ks, ds))
    return [int(x) for x in ks[order]]


def brute_min(A: int, B: int, N: int, M: int = M64):
    """Exact min over x < N of (B - x A) mod M and its smallest argmin."""
    best = None
    for x in range(N):
        d = (B - x * A) % M
        if best is None or d < best[0]:
            best = (d, x)
    return best


@dataclass
class LowerBound:
    success: bool          # True: certified no hit below the threshold
    d: int                 # distance value when the algorithm stopped
    u: int
    v: int
    iterations: int
    trace: list = field(default_factory=list)   # (d, p, q, u, v) after each iteration

    @property
    def ds(self):
        return [t[0] for t in self.trace]


# A two-length configuration (Sec. 3.2) is held as two sides: side 0 is the
# length p with its count u, side 1 the length q with its count v (the
# letters of Alg. 1-4).  Growing the configuration shortens one length by
# the other (the Euclidean recurrences behind Eq. 2 and Eq. 3): the side
# being shortened is called `r` below, the other one `o = 1 - r`.

def _shorten(L, C, r, counts_to_r):
    """Division-based step: L[r] loses floor(L[r] / L[o]) copies of L[o].

    Each removed copy adds intervals on the other side; the count that grows
    is C[r] (counts_to_r) or C[o], depending on which length each count is
    attached to in the caller's convention.  Returns the quotient.
    """
    o = 1 - r
    k = L[r] // L[o]
    L[r] -= k * L[o]
    if counts_to_r:
        C[r] += k * C[o]
    else:
        C[o] += k * C[r]
    return k


def _snapshot(d, L, C):
    return (d, L[0], L[1], C[0], C[1])


def lefevre_alg1(A: int, B: int, N: int, eps: int, M: int = M64):
    """Lefevre's lower bound computation and test, Alg. 1 (Sec. 4.1).

    Lengths p = {a} and q = 1 - {a} start with one interval each; d is the
    distance from {b} to the closest placed point on its left.  One round:
    if d >= p, a point has landed just left of b at distance p, so d drops
    by p (Failure as soon as d < eps) and the p side is the one shortened;
    otherwise the q side is.  The shortened side is first reduced by
    division (configuration (i, t) -> (i + 1, 0)), the run exits with
    Success once u + v >= N intervals exist, and then one subtraction step
    ((i + 1, 0) -> (i + 1, 1)) moves a point towards b.  A zero length
    means the points have become periodic (rational a): d is then final.
    """
    L, C = [A % M, M - A % M], [1, 1]
    d = B % M
    it = 0
    trace = []
    if d < eps:
        return LowerBound(False, d, C[0], C[1], it, trace)
    if L[0] == 0:   # every point sits at 0: d is already the exact minimum
        return LowerBound(True, d, C[0], C[1], it, trace)
    while True:
        it += 1
        r = 0 if d >= L[0] else 1
        if r == 0:
            d -= L[0]
            if d < eps:
                trace.append(_snapshot(d, L, C))
                return LowerBound(False, d, C[0], C[1], it, trace)
        if L[1 - r] == 0:
            if r == 0:
                trace.append(_snapshot(d, L, C))
            return LowerBound(d >= eps, d, C[0], C[1], it, trace)
        _shorten(L, C, r, counts_to_r=False)
        if C[0] + C[1] >= N:
            trace.append(_snapshot(d, L, C))
            return LowerBound(True, d, C[0], C[1], it, trace)
        # one subtraction: the other side loses the new length r once
        L[1 - r] -= L[r]
        C[r] += C[1 - r]
        trace.append(_snapshot(d, L, C))


def _regular_round(L, C, d, r, printed):
    """One partial quotient of the regular search (Alg. 2/4): the side r is
    shortened by division and d, b's distance to the closest point on its
    left, follows the split (Props. 1-2): after q shrinks, b's interval is
    cut at multiples of p; after p shrinks, b moves on only if it lies
    beyond the new p, and then modulo q.

    The counts follow Eq. 3 (v p + u q = 1 after every round) unless
    `printed`, which applies the updates as the listings print them."""
    _shorten(L, C, r, counts_to_r=not printed)
    if r == 1:
        return d % L[0]
    if d >= L[0]:
        return (d - L[0]) % L[1]
    return d


def regular_alg2(A: int, B: int, N: int, eps: int, M: int = M64,
                 printed: bool = False):
    """New regular lower bound computation and test, Alg. 2 (Sec. 4.2).

    Starting from p = {a}, q = 1 and one interval, each round completes one
    partial quotient of the continued fraction of a (division-based Euclid,
    configurations (i, 0) of Eq. 3): whichever of p and q is longer is
    shortened (see _regular_round).  Success iff d >= eps once the
    configuration holds u + v >= N intervals; a zero length (rational a,
    periodic points) ends the walk with d exact.
    """
    L, C = [A % M, M], [1, 0]
    d = B % M
    it = 0
    trace = []
    if d < eps:
        return LowerBound(False, d, C[0], C[1], it, trace)
    while True:
        r = 1 if L[0] < L[1] else 0
        if L[1 - r] == 0:
            return LowerBound(d >= eps, d, C[0], C[1], it, trace)
        it += 1
        d = _regular_round(L, C, d, r, printed)
        trace.append(_snapshot(d, L, C))
        if C[0] + C[1] >= N:
            return LowerBound(d >= eps, d, C[0], C[1], it, trace)


def regular_alg4(A: int, B: int, N: int, eps: int, M: int = M64,
                 printed: bool = False):
    """Regular test unrolled by two rounds, Alg. 4 (Sec. 4.3).

    In Alg. 2 the longer length alternates (q first, since p = {a} < 1), so
    the rounds run in fixed pairs, q side then p side, without comparing
    the lengths.
    """
    L, C = [A % M, M], [1, 0]
    d = B % M
    it = 0
    trace = []
    r = 1
    while True:
        if L[1 - r] == 0:
            return LowerBound(d >= eps, d, C[0], C[1], it, trace)
        it += r          # iterations count passes of the unrolled loop
        d = _regular_round(L, C, d, r, printed)
        trace.append(_snapshot(d, L, C))
        if C[0] + C[1] >= N:
            return LowerBound(d >= eps, d, C[0], C[1], it, trace)
        r = 1 - r
