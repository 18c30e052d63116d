"""HR cases: per-argument brute force and the three-phase pipeline oracle.

``hr_bruteforce`` is the plain definition (Def. 2-3 of the paper, Sec. 3.1):
evaluate f(X) at high precision for every binary64 argument and keep those
within eps ulp of a rounding breakpoint.  Feasible up to ~2^18 arguments.

``pipeline`` follows the paper's method on larger ranges (Sec. 3.1 steps,
Sec. 4.1 phases, Sec. 5 polynomial generation):

  * initial table of each sub-interval from its Taylor polynomial (taylor.py);
  * each piece's rows r_j(i) by the straightforward shift (tabulate.py);
  * phase 1: Lefevre's test (Alg. 1) on the piece's degree-1 truncation
    (Eq. 1) with a window widened by the truncation error of the piece, the
    approximation and rounding errors and the 64-bit truncation of (a, b);
  * phase 3: failing pieces are scanned exhaustively by tabulated
    differences (C, native.py) and every value is classified against the HR
    test with the same error margin;
  * values inside the margin are decided per argument by the brute force.

The paper's phase 2 (splitting failing pieces) only saves work; it is left
out so that the oracle stays plain.  The result is the set of argument
offsets m (X = X0 + m h) that are HR cases, sorted.
"""
from __future__ import annotations

from math import comb

import mpmath
import numpy as np
from mpmath import mpf

from . import native
from .search import lefevre_alg1
from .tabulate import piece_ab, straightforward_rows
from .taylor import (Job, arg_ulp, eps_approx, eps_round, f_value,
                     initial_table, out_ulp)

M64 = 1 << 64


def distance(job: Job, m: int, uf=None, prec: int = 192) -> mpf:
    """Distance of f(X)/u_f to the nearest breakpoint (Def. 2-3), X = X0 +
    m h: to the nearest midpoint (Z + 1/2) in round-to-nearest mode, to
    the nearest integer (representable number) in directed mode.  Computed
    at `prec` bits; the caller keeps the mpmath context of that precision
    to use it."""
    uf = out_ulp(job) if uf is None else uf
    with mpmath.workprec(prec):
        X = mpf(job.X0) + m * arg_ulp(job.X0)
        y = f_value(job.fname, X) / uf
        z = y - (mpf(1) / 2 if job.mode == "rn" else 0)
        return abs(z - mpmath.nint(z))


def _is_hr(job: Job, m: int, uf, prec: int) -> bool:
    eps = mpf(2) ** (-job.s)
    with mpmath.workprec(prec):
        dist = distance(job, m, uf, prec)
        if abs(dist - eps) < mpf(2) ** (-(prec - 64)):
            if prec > 4096:
                raise ArithmeticError("distance equals eps to 4096 bits")
            return _is_hr(job, m, uf, 2 * prec)
        return dist < eps


def hr_bruteforce(job: Job, start: int = 0, count: int | None = None, prec: int = 192):
    """Offsets m in [start, start + count) whose argument is a (53, 2^-s) HR case."""
    count = job.count - start if count is None else count
    uf = out_ulp(job)
    return [m for m in range(start, start + count) if _is_hr(job, m, uf, prec)]


def decide(job: Job, m: int) -> bool:
    """Exact HR decision for one argument offset (used for undecided values)."""
    return _is_hr(job, m, out_ulp(job), 192)


def _centered(x: int, W: int) -> int:
    return x - (1 << W) if x >= (1 << (W - 1)) else x


def piece_window(rows, job: Job, mu):
    """(LO, D) of the widened degree-1 window of one piece, integers mod 2^64.

    Truncation term sum_{j>=2} r_j C(x, j), x < N, is bounded by the piece's
    own rows (centred representatives are the true small values).
    """
    W = job.W
    tb = sum(abs(_centered(rows[j], W)) * comb(job.N - 1, j)
             for j in range(2, job.delta + 1))
    with mpmath.workprec(W + 128):
        Tb = mpf(tb) / mpf(2) ** W
        eps = mpf(2) ** (-job.s)
        one = mpf(2) ** (-64)
        lo = -(mu + Tb + one)
        D = 2 * eps + 2 * mu + 2 * Tb + (job.N + 1) * one
        LO = int(mpmath.floor(lo * mpf(2) ** 64)) % M64
        Dint = min(int(mpmath.ceil(D * mpf(2) ** 64)) + 2, M64 - 1)
    return LO, Dint


def value_thresholds(job: Job, mu):
    """Integer thresholds on the top 64 bits t of a piece value (see module doc)."""
    with mpmath.workprec(256):
        eps = mpf(2) ** (-job.s)
        s64 = mpf(2) ** 64
        hr_lo = int(mpmath.ceil(mu * s64))
        hr_hi = int(mpmath.floor((2 * eps - mu) * s64)) - 1
        rej_lo = int(mpmath.ceil((2 * eps + mu) * s64))
        rej_hi = int(mpmath.floor((1 - mu) * s64)) - 1
    return hr_lo, hr_hi, rej_lo, rej_hi


def pipeline(job: Job, subs=None, pieces=None, use_filter: bool = True,
             threads: int | None = None, stats: dict | None = None):
    """HR offsets of the job (or of the chosen sub-intervals / pieces).

    subs: iterable of sub-interval indices (default: all); pieces: iterable of
    piece indices inside each sub-interval (default: all tau).
    """
    W, d, N = job.W, job.delta, job.N
    L = W // 64
    subs = range(job.n_sub) if subs is None else subs
    pieces = list(range(job.tau)) if pieces is None else list(pieces)
    out = []
    st = {"pieces": 0, "phase3_pieces": 0, "sure": 0, "undecided": 0}
    for t in subs:
        T = initial_table(job, t)
        with mpmath.workprec(128):
            mu = eps_approx(job, t) + eps_round(job)
        thr = value_thresholds(job, mu)
        fail_rows, fail_base = [], []
        for i in pieces:
            st["pieces"] += 1
            rows = straightforward_rows(T, d, i, W)
            if use_filter:
                a, b = piece_ab(rows, W)
                LO, D = piece_window(rows, job, mu)
                if lefevre_alg1(a, (b - LO) % M64, N, D).success:
                    continue
            fail_rows.append([[(r >> (64 * l)) & (M64 - 1) for l in range(L)] for r in rows])
            fail_base.append(t * job.per_sub + i * N)
        st["phase3_pieces"] += len(fail_rows)
        if not fail_rows:
            continue
        n = len(fail_rows)
        rows_np = np.array(fail_rows, dtype=np.uint64).reshape(n, d + 1, L)
        full = lambda v: np.full(n, v, np.uint64)
        counts, xs, cls = native.exhaustive_many(
            rows_np, np.full(n, N, np.uint32), full(thr[0]), full(thr[1]),
            full(thr[2]), full(thr[3]), d, L, threads)
        pos = 0
        for p in range(n):
            for j in range(int(counts[p])):
                m = fail_base[p] + int(xs[pos])
                if cls[pos] == 1:
                    st["sure"] += 1
                    out.append(m)
                else:
                    st["undecided"] += 1
                    if decide(job, m):
                        out.append(m)
                pos += 1
    if stats is not None:
        stats.update(st)
    return sorted(out)
