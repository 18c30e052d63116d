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


def lefevre_alg1(A: int, B: int, N: int, eps: int, M: int = M64):
    """Lefevre's lower bound computation and test, Alg. 1 (Sec. 4.1).

    p, q hold the two interval lengths, u, v their counts (u p + v q = 1,
    Eq. 2), d the distance from b to the closest point on its left.  The
    first branch reduces the length not containing b by division; the
    second moves one point to the left of b by subtraction.  Returns on
    u + v >= N (Success) or when d drops below eps (Failure: a point with
    index < N lies within eps to the left of b).
    """
    p = A % M
    q = M - p
    d = B % M
    u, v = 1, 1
    it = 0
    trace = []
    if d < eps:
        return LowerBound(False, d, u, v, it, trace)
    if p == 0:   # every point sits at 0: d is already the exact minimum
        return LowerBound(True, d, u, v, it, trace)
    while True:
        it += 1
        if d < p:
            if p == 0:
                return LowerBound(d >= eps, d, u, v, it, trace)
            k = q // p
            q -= k * p
            u += k * v
            if u + v >= N:
                trace.append((d, p, q, u, v))
                return LowerBound(True, d, u, v, it, trace)
            p -= q
            v += u
        else:
            d -= p
            if d < eps:
                trace.append((d, p, q, u, v))
                return LowerBound(False, d, u, v, it, trace)
            if q == 0:
                trace.append((d, p, q, u, v))
                return LowerBound(True, d, u, v, it, trace)
            k = p // q
            p -= k * q
            v += k * u
            if u + v >= N:
                trace.append((d, p, q, u, v))
                return LowerBound(True, d, u, v, it, trace)
            q -= p
            u += v
        trace.append((d, p, q, u, v))


def regular_alg2(A: int, B: int, N: int, eps: int, M: int = M64,
                 printed: bool = False):
    """New regular lower bound computation and test, Alg. 2 (Sec. 4.2).

    Each iteration completes one partial quotient of the continued fraction
    of a (division-based Euclid only, configurations (i, 0) of Eq. 3): the
    shorter length reduces the longer one, and d is reduced modulo the new
    length (Props. 1-2 give the side on which intervals split).  Returns
    Success iff d >= eps once u + v >= N.
    """
    p = A % M
    q = M
    d = B % M
    u, v = 1, 0
    it = 0
    trace = []
    if d < eps:
        return LowerBound(False, d, u, v, it, trace)
    while True:
        if p < q:
            if p == 0:
                return LowerBound(d >= eps, d, u, v, it, trace)
            it += 1
            k = q // p
            q -= k * p
            if printed:
                u += k * v
            else:
                v += k * u
            d %= p
        else:
            if q == 0:
                return LowerBound(d >= eps, d, u, v, it, trace)
            it += 1
            k = p // q
            p -= k * q
            if printed:
                v += k * u
            else:
                u += k * v
            if d >= p:
                d = (d - p) % q
        trace.append((d, p, q, u, v))
        if u + v >= N:
            return LowerBound(d >= eps, d, u, v, it, trace)


def regular_alg4(A: int, B: int, N: int, eps: int, M: int = M64,
                 printed: bool = False):
    """Regular test unrolled by two iterations, Alg. 4 (Sec. 4.3).

    Alg. 2's condition p < q alternates deterministically (true first, since
    p starts at {a} and q at 1), so two half-steps per loop need no test on
    which length to reduce.
    """
    p = A % M
    q = M
    d = B % M
    u, v = 1, 0
    it = 0
    trace = []
    while True:
        if p == 0:
            return LowerBound(d >= eps, d, u, v, it, trace)
        it += 1
        k = q // p
        q -= k * p
        if printed:
            u += k * v
        else:
            v += k * u
        d %= p
        trace.append((d, p, q, u, v))
        if u + v >= N:
            return LowerBound(d >= eps, d, u, v, it, trace)
        if q == 0:
            return LowerBound(d >= eps, d, u, v, it, trace)
        k = p // q
        p -= k * q
        if printed:
            v += k * u
        else:
            u += k * v
        if d >= p:
            d = (d - p) % q
        trace.append((d, p, q, u, v))
        if u + v >= N:
            return LowerBound(d >= eps, d, u, v, it, trace)
