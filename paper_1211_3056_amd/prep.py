"""Host preparation of HR-case search jobs.

A job searches the binary64 arguments X0 + m h, 0 <= m < count, of f for
round-to-nearest (or directed) hard-to-round cases at distance below
eps = 2^-s output ulps (Sec. 3.1 of the paper: change of variable to integer
arguments, HR test {y - c + eps} < 2 eps with c = 1/2 for nearest, 0 for
directed).  The range is cut into sub-intervals of tau * N arguments and
each sub-interval into tau pieces of N (Sec. 5, hierarchical method).

For every sub-interval this module produces what the device path consumes:

* the initial table T[j][l] = Delta_N^l Delta_1^j R(0) (j + l <= delta) of the
  degree-delta Taylor polynomial R of f(X_t + x h)/u_f - c + eps, rounded
  once to W-bit fractions.  R is held by its monomial coefficients c_n as
  fixed-point integers with guard bits; the table is their image under the
  exact integer matrices K_n[j][l] = Delta_N^l Delta_1^j (x^n)(0);
* the degree-1 window (lo, d): every argument whose value can pass the HR
  test has (b - lo - k a) mod 2^64 < d.  It covers the truncation to degree
  one (bounded through interval bounds on R's derivatives, one-sided when
  their sign is fixed), the approximation and rounding errors, and the
  64-bit truncation of a and b;
* the thresholds (hr_lo, hr_hi, rej_lo, rej_hi) on the top 64 bits of an
  exact piece value: certainly HR, certainly not, or undecided (decided
  here at high precision by ``decide``).

Transcendental values come from mpmath at W + guard + 64 bits.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass
from math import comb

import mpmath
import numpy as np
from mpmath import mpf

M64 = 1 << 64
FUNCTIONS = ("exp", "exp2", "log", "sin", "cos")


@dataclass(frozen=True)
class JobSpec:
    fname: str
    X0: float
    count: int
    s: int                 # eps = 2^-s output ulps
    mode: str = "rn"       # "rn" or "dir"
    N: int = 1 << 16
    tau: int = 1 << 8
    delta: int = 3
    W: int = 192

    @property
    def per_sub(self) -> int:
        return self.N * self.tau

    @property
    def n_sub(self) -> int:
        if self.count % self.per_sub:
            raise ValueError("count must be a multiple of N * tau")
        return self.count // self.per_sub

    @property
    def limbs(self) -> int:
        return self.W // 64

    @property
    def entries(self) -> int:
        return (self.delta + 1) * (self.delta + 2) // 2


def _ulp(x) -> mpf:
    """ulp of a binary64 number with x = m 2^e, m in [1/2, 1): 2^(e-53)."""
    _, e = mpmath.frexp(mpf(x))
    return mpf(2) ** (e - 53)


def _f(fname, X):
    if fname == "exp":
        return mpmath.exp(X)
    if fname == "exp2":
        return mpmath.power(2, X)
    if fname == "log":
        return mpmath.log(X)
    if fname == "sin":
        return mpmath.sin(X)
    if fname == "cos":
        return mpmath.cos(X)
    raise ValueError(fname)


def _taylor_coeffs(fname, X, n_max, h, uf):
    """f^(n)(X) h^n / (n! u_f), n <= n_max, at the current precision."""
    out = []
    if fname == "exp":
        e = mpmath.exp(X)
        t = e / uf
        for n in range(n_max + 1):
            out.append(t)
            t = t * h / (n + 1)
        return out
    if fname == "exp2":
        e = mpmath.power(2, X)
        l2 = mpmath.ln2
        t = e / uf
        for n in range(n_max + 1):
            out.append(t)
            t = t * l2 * h / (n + 1)
        return out
    if fname == "log":
        out.append(mpmath.log(X) / uf)
        for n in range(1, n_max + 1):
            # log^(n)(X)/n! = (-1)^(n-1) / (n X^n)
            out.append((-1) ** (n - 1) * (h / X) ** n / (n * uf))
        return out
    if fname in ("sin", "cos"):
        s, c = mpmath.sin(X), mpmath.cos(X)
        cyc = [s, c, -s, -c] if fname == "sin" else [c, -s, -c, s]
        fact = mpf(1)
        for n in range(n_max + 1):
            if n:
                fact *= n
            out.append(cyc[n % 4] * h ** n / (fact * uf))
        return out
    raise ValueError(fname)


def _deriv_bound(fname, X_lo, X_hi, n):
    """max |f^(n)| on [X_lo, X_hi] from closed forms (monotone or bounded)."""
    if fname == "exp":
        return mpmath.exp(X_hi)
    if fname == "exp2":
        return mpmath.ln2 ** n * mpmath.power(2, X_hi)
    if fname == "log":
        return mpmath.factorial(n - 1) / X_lo ** n
    return mpf(1)


def _k_matrices(N: int, delta: int):
    """K[n][(j, l)] = Delta_N^l Delta_1^j (x^n) at 0, exact integers."""
    K = []
    for n in range(delta + 1):
        Kn = {}
        for j in range(delta + 1):
            for l in range(delta - j + 1):
                acc = 0
                for s in range(l + 1):
                    for m in range(j + 1):
                        sign = -1 if (l - s + j - m) & 1 else 1
                        acc += sign * comb(l, s) * comb(j, m) * (s * N + m) ** n
                Kn[(j, l)] = acc
        K.append(Kn)
    return K


def round_bound(N: int, tau: int, delta: int, W: int) -> mpf:
    """Bound on how far rounding the table entries to W bits moves a piece
    value.  Every entry T[j][l] (j + l <= delta) is within 2^-(W+1) of its
    exact value (the fixed-point monomials carry guard bits, so their own
    error is far smaller); the value of piece i at x is
    sum_{j+l<=delta} T[j][l] C(i, l) C(x, j) (Sec. 5.1-5.2), whose
    binomials peak at i = tau - 1, x = N - 1.  Twice that maximum:
    2^-W sum_{j+l<=delta} C(N-1, j) C(tau-1, l)."""
    return mpf(2) ** (-W) * round_sum(N, tau, delta)


def round_sum(N: int, tau: int, delta: int) -> int:
    """sum_{j+l<=delta} C(N-1, j) C(tau-1, l), the integer factor of round_bound."""
    return sum(comb(N - 1, j) * comb(tau - 1, l)
               for j in range(delta + 1) for l in range(delta - j + 1))


@dataclass
class Prepared:
    spec: JobSpec
    subs: np.ndarray        # sub-interval indices covered, int64
    tables: np.ndarray      # uint64 (n, E, L)
    win: np.ndarray         # uint64 (n, 2): lo, d
    thr: np.ndarray         # uint64 (n, 4): hr_lo, hr_hi, rej_lo, rej_hi
    h: mpf
    uf: mpf


@functools.lru_cache(maxsize=4096)
def output_ulp_range(fname: str, X0: float, count: int) -> mpf:
    """ulp of f on [X0, X0 + count h); f must stay in one binade there
    (memoised: a job's preparation asks for it more than once)."""
    with mpmath.workprec(128):
        h = _ulp(X0)
        lo = _f(fname, mpf(X0))
        hi = _f(fname, mpf(X0) + (count - 1) * h)
        e1, e2 = mpmath.frexp(lo)[1], mpmath.frexp(hi)[1]
        if e1 != e2 or lo <= 0:
            raise ValueError(f"{fname} leaves its output binade on this range")
        return mpf(2) ** (e1 - 53)


def output_ulp(spec: JobSpec) -> mpf:
    return output_ulp_range(spec.fname, spec.X0, spec.count)


class SubPreparer:
    """Tables, windows and thresholds of sub-intervals of one function range.

    A sub-interval starts `start` arguments after X0, holds `length`
    arguments and is cut into pieces of N arguments (the last one partial
    when N does not divide length).  Its polynomial is the degree-delta
    Taylor expansion at its first argument.
    """

    def __init__(self, fname: str, X0: float, s: int, mode: str, delta: int, W: int, uf):
        if fname not in FUNCTIONS:
            raise ValueError(fname)
        if W not in (128, 192, 256) or not 1 <= delta <= 6:
            raise ValueError("unsupported width or degree")
        self.fname, self.X0, self.s, self.mode = fname, X0, s, mode
        self.delta, self.W, self.uf = delta, W, uf
        self.pairs = [(j, l) for j in range(delta + 1) for l in range(delta - j + 1)]
        self._K = {}

    def _kmat(self, N):
        if N not in self._K:
            K = _k_matrices(N, self.delta)
            kmax = max(abs(v) for Kn in K for v in Kn.values())
            self._K[N] = (K, kmax.bit_length() + 96)
        return self._K[N]

    def prepare(self, start: int, length: int, N: int):
        """(table uint64 (E, L), window uint64 (2,), thresholds uint64 (4,))."""
        d, W = self.delta, self.W
        L = W // 64
        tau = -(-length // N)
        K, G = self._kmat(N)
        table = np.zeros((len(self.pairs), L), np.uint64)
        win = np.zeros(2, np.uint64)
        thr = np.zeros(4, np.uint64)
        with mpmath.workprec(W + G + 64):
            h = _ulp(self.X0)
            uf = self.uf
            eps = mpf(2) ** (-self.s)
            Xt = mpf(self.X0) + start * h
            c = _taylor_coeffs(self.fname, Xt, d, h, uf)
            c[0] += eps - (mpf(1) / 2 if self.mode == "rn" else 0)
            scale = mpf(2) ** (W + G)
            C = [int(mpmath.nint(cn * scale)) for cn in c]
            for e, (j, l) in enumerate(self.pairs):
                v = sum(C[n] * K[n][(j, l)] for n in range(d + 1))
                v = ((v + (1 << (G - 1))) >> G) & ((1 << W) - 1)
                for li in range(L):
                    table[e, li] = (v >> (64 * li)) & (M64 - 1)
            # error budget of this sub-interval
            M = length
            e_round = round_bound(N, tau, d, W)
            e_row = mpf(2) ** (-W - 1) * sum(comb(tau - 1, l) for l in range(d + 1))
            nA = d + 1
            e_approx = _deriv_bound(self.fname, Xt, Xt + M * h, nA) * (M * h) ** nA \
                / (mpmath.factorial(nA) * uf) * mpf("1.01")
            mu = e_approx + e_round
            # r_j(i) = Delta^j R(i N) lies in the range of R^(j) on [0, M + d]
            Y = mpf(M + d)
            t_lo = t_hi = mpf(0)
            for j in range(2, d + 1):
                lo_j = hi_j = c[j] * mpmath.factorial(j)
                for n in range(j + 1, d + 1):
                    term = c[n] * mpmath.factorial(n) / mpmath.factorial(n - j) * Y ** (n - j)
                    lo_j += min(term, 0)
                    hi_j += max(term, 0)
                cj = comb(N - 1, j)
                t_lo += min(lo_j - e_row, 0) * cj
                t_hi += max(hi_j + e_row, 0) * cj
            one = mpf(2) ** -64
            lo = -(mu + t_hi + one)
            width = 2 * eps + 2 * mu + (t_hi - t_lo) + (N + 1) * one
            s64 = mpf(2) ** 64
            win[0] = int(mpmath.floor(lo * s64)) % M64
            win[1] = min(int(mpmath.ceil(width * s64)) + 2, M64 - 1)
            thr[:] = value_bands(mu, eps)
        return table, win, thr


def value_bands(mu, eps):
    """(hr_lo, hr_hi, rej_lo, rej_hi) on the top 64 bits t of an exact piece
    value v = y - c + eps + e, |e| <= mu: HR for sure iff
    mu <= t 2^-64 and t 2^-64 + 2^-64 <= 2 eps - mu, rejected for sure iff
    2 eps + mu <= t 2^-64 and t 2^-64 + 2^-64 <= 1 - mu.  When the error
    budget leaves no room for a band (mu too large for eps, a degree or
    width too small for the job), that band is empty (lo = 2^64 - 1 > hi =
    0): every candidate is then undecided and decided on the host."""
    s64 = mpf(2) ** 64
    hr_lo = int(mpmath.ceil(mu * s64))
    hr_hi = int(mpmath.floor((2 * eps - mu) * s64)) - 1
    rej_lo = int(mpmath.ceil((2 * eps + mu) * s64))
    rej_hi = int(mpmath.floor((1 - mu) * s64)) - 1
    out = []
    for lo, hi in ((hr_lo, hr_hi), (rej_lo, rej_hi)):
        if hi < lo or lo > M64 - 1 or hi < 0:
            lo, hi = M64 - 1, 0
        out += [max(lo, 0), min(hi, M64 - 1)]
    return out


def _prepare_rows(spec: JobSpec, subs: np.ndarray, uf):
    sp = SubPreparer(spec.fname, spec.X0, spec.s, spec.mode, spec.delta, spec.W, uf)
    tables = np.zeros((len(subs), spec.entries, spec.limbs), np.uint64)
    win = np.zeros((len(subs), 2), np.uint64)
    thr = np.zeros((len(subs), 4), np.uint64)
    for row, t in enumerate(subs):
        tables[row], win[row], thr[row] = sp.prepare(int(t) * spec.per_sub, spec.per_sub, spec.N)
    return tables, win, thr


def _prepare_chunk(args):
    spec, subs, uf = args
    return _prepare_rows(spec, subs, uf)


def prepare(spec: JobSpec, subs=None, pool=None) -> Prepared:
    """Tables, windows and thresholds for the given sub-intervals (default
    all).  pool: an optional process pool (concurrent.futures); the
    sub-intervals are then prepared in chunks by its workers.  The result
    does not depend on the pool."""
    subs = np.arange(spec.n_sub, dtype=np.int64) if subs is None else np.asarray(subs, np.int64)
    uf = output_ulp(spec)
    workers = getattr(pool, "_max_workers", 0) if pool is not None else 0
    if workers > 1 and len(subs) >= 2 * workers:
        chunks = np.array_split(subs, 4 * workers)
        parts = list(pool.map(_prepare_chunk, [(spec, c, uf) for c in chunks if len(c)]))
        tables, win, thr = (np.concatenate([p[i] for p in parts]) for i in range(3))
    else:
        tables, win, thr = _prepare_rows(spec, subs, uf)
    with mpmath.workprec(64):
        h = _ulp(spec.X0)
    return Prepared(spec, subs, tables, win, thr, h, uf)


def is_hr(spec: JobSpec, m: int, uf=None, prec: int = 192) -> bool:
    """Exact decision for one argument offset m (high-precision evaluation)."""
    uf = output_ulp(spec) if uf is None else uf
    with mpmath.workprec(prec):
        X = mpf(spec.X0) + m * _ulp(spec.X0)
        y = _f(spec.fname, X) / uf
        if spec.mode == "rn":
            y -= mpf(1) / 2
        dist = abs(y - mpmath.nint(y))
        eps = mpf(2) ** (-spec.s)
        if abs(dist - eps) < mpf(2) ** (64 - prec):
            if prec >= 4096:
                raise ArithmeticError("undecidable at 4096 bits")
            return is_hr(spec, m, uf, 2 * prec)
        return bool(dist < eps)


# ---------------------------------------------------------------- upper level
#
# The top of the hierarchical method (Sec. 5.1): one polynomial U of higher
# degree Du for a whole range, tabulated once on the host into its
# hierarchical table with steps 1 and S (S = arguments per sub-interval);
# the device turns it into every sub-interval's initial table (hr_subtables:
# straightforward shift in the sub-interval index, Sec. 5.2, then the
# sub-interval's table with steps 1 and N, truncated to degree delta and
# rounded to W bits).  Only the upper table, one window and one set of
# thresholds per piece length are made here, in place of one Taylor
# expansion per sub-interval.

UPPER_WIDTHS = (192, 256, 320, 384, 448)
MAX_UPPER_DEGREE = 10           # HR_MAX_UPPER_DEGREE of include/hrsearch.h


_KCACHE: dict = {}


def _kmat_cached(S: int, Du: int):
    key = (S, Du)
    if key not in _KCACHE:
        K = _k_matrices(S, Du)
        kmax = max(abs(v) for Kn in K for v in Kn.values())
        pairs = [(n, m) for n in range(Du + 1) for m in range(Du - n + 1)]
        cols = [[(k, K[k][p]) for k in range(Du + 1) if K[k][p]] for p in pairs]
        _KCACHE[key] = (K, kmax.bit_length() + 96, cols)
    return _KCACHE[key]


@dataclass
class UpperTable:
    fname: str
    X0: float
    count: int
    s: int
    mode: str
    S: int                 # arguments per sub-interval (step of the table in x)
    Du: int                # degree of U
    Wu: int                # word width of the table entries
    words: np.ndarray      # uint64 (E_u, Wu/64): entry (n, m) = Delta_S^m Delta_1^n U(0)
    coeffs: list           # monomial coefficients of U (mpf), -c + eps folded into c_0
    uf: object
    e_approx: object       # |U(x) - g(x)| over the range (Lagrange remainder)

    @property
    def n_sub(self) -> int:
        return -(-self.count // self.S)

    def shift_error(self, n: int):
        """Bound on the error of Delta_1^n R_t(0) = sum_m U[n][m] C(t, m) for
        any sub-interval t < n_sub, from the rounding of U's entries to Wu
        bits (twice 2^-(Wu+1), covering the guard bits' own error)."""
        T = self.n_sub
        return mpf(2) ** (-self.Wu) * sum(comb(T - 1, m) for m in range(self.Du - n + 1))


@functools.lru_cache(maxsize=4096)
def upper_error(fname: str, X0: float, count: int, Du: int, uf) -> mpf:
    """Lagrange remainder of the degree-Du Taylor polynomial at X0 over the
    whole range [X0, X0 + count h), in output ulps (closed-form bounds of
    |f^(Du+1)|), with a 1% margin."""
    with mpmath.workprec(128):
        h = _ulp(X0)
        n = Du + 1
        return _deriv_bound(fname, mpf(X0), mpf(X0) + count * h, n) * (count * h) ** n \
            / (mpmath.factorial(n) * uf) * mpf("1.01")


def upper_table(fname: str, X0: float, count: int, s: int, mode: str, S: int, Du: int,
                Wu: int, uf=None) -> UpperTable:
    """Upper table of the range [X0, X0 + count h): the hierarchical table,
    steps 1 and S, of the degree-Du Taylor polynomial U of
    g(x) = f(X0 + x h)/u_f - c + eps at x = 0, each entry rounded once to
    the nearest Wu-bit fraction (exact integer image of fixed-point
    monomial coefficients, as for the sub-interval tables)."""
    if fname not in FUNCTIONS or Wu not in UPPER_WIDTHS or not 1 <= Du <= MAX_UPPER_DEGREE:
        raise ValueError("unsupported function, upper width or upper degree")
    uf = output_ulp_range(fname, X0, count) if uf is None else uf
    K, G, cols = _kmat_cached(S, Du)
    pairs = [(n, m) for n in range(Du + 1) for m in range(Du - n + 1)]
    Lw = Wu // 64
    words = np.zeros((len(pairs), Lw), np.uint64)
    with mpmath.workprec(Wu + G + 64):
        h = _ulp(X0)
        eps = mpf(2) ** (-s)
        c = _taylor_coeffs(fname, mpf(X0), Du, h, uf)
        c[0] += eps - (mpf(1) / 2 if mode == "rn" else 0)
        scale = mpf(2) ** (Wu + G)
        C = [int(mpmath.nint(cn * scale)) for cn in c]
    mask = (1 << Wu) - 1
    for e, col in enumerate(cols):
        v = sum(C[k] * kv for k, kv in col)
        v = ((v + (1 << (G - 1))) >> G) & mask
        for li in range(Lw):
            words[e, li] = (v >> (64 * li)) & (M64 - 1)
    return UpperTable(fname, X0, count, s, mode, S, Du, Wu, words, c, uf,
                      upper_error(fname, X0, count, Du, uf))


def upper_windows_precise(U: UpperTable, N: int, tau: int, delta: int, W: int):
    """Degree-1 window (lo, d), thresholds and error bound mu of every
    sub-interval of the range whose table the device makes from U with
    pieces of N arguments, tau pieces, degree delta and width W.

    Write R_t(y) = U(t S + y) and R~_t = R_t + E_t for the polynomial the
    device shifts out of the rounded upper table (E_t(y) = sum_n e_n C(y, n),
    |e_n| <= U.shift_error(n)).  The sub-interval table keeps the entries
    j + l <= delta of R~_t's table with steps 1 and N and rounds them to W
    bits, so a piece value differs from g by at most
      mu = e_approx(U)                                  (Lagrange remainder)
         + sum_{j+l>delta} N^l max|U^(j+l)| C(tau-1, l) C(N-1, j)
                                                        (dropped entries of R_t)
         + sum_{j+l<=delta} |Delta_N^l Delta_1^j E_t(0)| C(tau-1, l) C(N-1, j)
                                                        (kept entries of E_t)
         + 2^-W sum_{j+l<=delta} C(N-1, j) C(tau-1, l)  (rounding to W bits),
    using Delta_N^l Delta_1^j R_t(0) = N^l U^(j+l)(xi) (mean value form of
    differences) and |Delta_N^l C(y, n-j)| <= 2^l C(l N, n-j) at 0.  The terms
    r_j C(x, j), j >= 2, of the degree-1 window are bounded through the range
    of U^(j) on the job's offsets plus the same dropped, shifted and
    rounding parts of row j."""
    d = delta
    if not 1 <= d <= min(U.Du, 8):
        raise ValueError("degree must be between 1 and the upper degree")
    with mpmath.workprec(192):
        c = U.coeffs
        Du = U.Du
        eps = mpf(2) ** (-U.s)
        X = mpf(U.count + d * N + d)            # largest offset a difference reaches
        fac = mpmath.factorial

        def dmax(n):                            # max |U^(n)(x)|, 0 <= x <= X
            return sum(abs(c[k]) * fac(k) / fac(k - n) * X ** (k - n) for k in range(n, Du + 1))

        def drange(j):                          # range of U^(j) on [0, X]
            lo = hi = c[j] * fac(j)
            for k in range(j + 1, Du + 1):
                term = c[k] * fac(k) / fac(k - j) * X ** (k - j)
                lo += min(term, 0)
                hi += max(term, 0)
            return lo, hi

        Mx = [dmax(n) for n in range(Du + 1)]
        en = [U.shift_error(n) for n in range(Du + 1)]
        drop = {}                               # |T[j][l]| of R_t, j + l > delta
        keptE = {}                              # |Delta_N^l Delta_1^j E_t(0)|, j + l <= delta
        for j in range(Du + 1):
            for l in range(Du - j + 1):
                if j + l > d:
                    drop[(j, l)] = mpf(N) ** l * Mx[j + l]
                else:
                    keptE[(j, l)] = sum(en[n] * 2 ** l * comb(l * N, n - j)
                                        for n in range(j + l, Du + 1))
        e_drop = sum(v * comb(tau - 1, l) * comb(N - 1, j) for (j, l), v in drop.items())
        e_shift = sum(v * comb(tau - 1, l) * comb(N - 1, j) for (j, l), v in keptE.items())
        e_rw = round_bound(N, tau, d, W)
        mu = U.e_approx + e_drop + e_shift + e_rw
        t_lo = t_hi = mpf(0)
        for j in range(2, d + 1):
            lo_j, hi_j = drange(j)
            slack = sum(drop[(j, l)] * comb(tau - 1, l) for l in range(d - j + 1, Du - j + 1)) \
                + sum(keptE[(j, l)] * comb(tau - 1, l) for l in range(d - j + 1)) \
                + mpf(2) ** (-W - 1) * sum(comb(tau - 1, l) for l in range(d - j + 1))
            cj = comb(N - 1, j)
            t_lo += min(lo_j - slack, 0) * cj
            t_hi += max(hi_j + slack, 0) * cj
        one = mpf(2) ** -64
        lo = -(mu + t_hi + one)
        width = 2 * eps + 2 * mu + (t_hi - t_lo) + (N + 1) * one
        s64 = mpf(2) ** 64
        win = np.array([int(mpmath.floor(lo * s64)) % M64,
                        min(int(mpmath.ceil(width * s64)) + 2, M64 - 1)], np.uint64)
        thr = np.array(value_bands(mu, eps), np.uint64)
    return win, thr, mu


_UP = 1.0 + 2.0 ** -40          # covers the rounding of the float sums below


_WCONST: dict = {}


def _window_consts(Du: int, Wu: int, n_sub: int, N: int, tau: int, d: int, W: int):
    """The parts of upper_windows that do not depend on the function: the
    binomial factors, the shift errors' kept entries and the rounding bound
    (floats with the same outward margins), cached per job shape."""
    key = (Du, Wu, n_sub, N, tau, d, W)
    if key not in _WCONST:
        T = n_sub
        en = [float(mpf(2) ** (-Wu) * sum(comb(T - 1, m) for m in range(Du - n + 1))) * _UP
              for n in range(Du + 1)]
        cN = [float(comb(N - 1, j)) * _UP for j in range(Du + 1)]
        cT = [float(comb(tau - 1, l)) * _UP for l in range(Du + 1)]
        keptE = {}
        for j in range(Du + 1):
            for l in range(Du - j + 1):
                if j + l <= d:
                    keptE[(j, l)] = sum(en[n] * 2.0 ** l * float(comb(l * N, n - j)) * _UP
                                        for n in range(j + l, Du + 1)) * _UP
        e_shift = sum(v * cT[l] * cN[j] for (j, l), v in keptE.items()) * _UP
        e_rw = float(round_bound(N, tau, d, W)) * _UP
        kept_slack = [(sum(keptE[(j, l)] * cT[l] for l in range(d - j + 1)),
                       2.0 ** (-W - 1) * sum(cT[l] for l in range(d - j + 1))) if j <= d
                      else (0.0, 0.0) for j in range(Du + 1)]
        _WCONST[key] = (cN, cT, e_shift, e_rw, kept_slack)
    return _WCONST[key]


def upper_windows(U: UpperTable, N: int, tau: int, delta: int, W: int):
    """The bounds of upper_windows_precise in binary64 arithmetic (a few
    hundred float operations instead of mpmath ones, for host preparation
    in well under a millisecond).  Every quantity is a sum of products of
    magnitudes (or, for the ranges of U^(j), a signed sum), evaluated with
    relative error far below 2^-40 and then pushed outwards by 2^-40 of its
    magnitude; the window and thresholds come from those outer bounds in
    exact integer arithmetic, so they contain the precise ones."""
    d = delta
    if not 1 <= d <= min(U.Du, 8):
        raise ValueError("degree must be between 1 and the upper degree")
    Du = U.Du
    cN, cT, e_shift, e_rw, kept_slack = _window_consts(Du, U.Wu, U.n_sub, N, tau, d, W)
    c = [float(x) for x in U.coeffs]
    ca = [abs(x) * _UP for x in c]
    X = float(U.count + d * N + d)
    fac = [float(math.factorial(k)) for k in range(Du + 1)]
    Xp = [X ** e * _UP for e in range(Du + 1)]
    Mx = [sum(ca[k] * fac[k] / fac[k - n] * Xp[k - n] for k in range(n, Du + 1)) * _UP
          for n in range(Du + 1)]
    drop = {}
    for j in range(Du + 1):
        for l in range(Du - j + 1):
            if j + l > d:
                drop[(j, l)] = float(N) ** l * Mx[j + l] * _UP
    e_drop = sum(v * cT[l] * cN[j] for (j, l), v in drop.items()) * _UP
    mu = (float(U.e_approx) * _UP + e_drop + e_shift + e_rw) * _UP
    t_lo = t_hi = 0.0
    for j in range(2, d + 1):
        base = c[j] * fac[j]
        lo_j = hi_j = base
        mag = abs(base)
        for k in range(j + 1, Du + 1):
            term = c[k] * fac[k] / fac[k - j] * X ** (k - j)
            lo_j += min(term, 0.0)
            hi_j += max(term, 0.0)
            mag += abs(term)
        slack = (sum(drop[(j, l)] * cT[l] for l in range(d - j + 1, Du - j + 1))
                 + kept_slack[j][0] + kept_slack[j][1]) * _UP
        margin = mag * 2.0 ** -40 + slack
        t_lo += min(lo_j - margin, 0.0) * cN[j] * _UP
        t_hi += max(hi_j + margin, 0.0) * cN[j] * _UP
    t_lo *= _UP
    t_hi *= _UP
    mu64 = math.ceil(mu * 2.0 ** 64)
    hi64 = math.ceil(t_hi * 2.0 ** 64)
    lo64 = math.floor(t_lo * 2.0 ** 64)
    e2 = 1 << (65 - U.s)                      # 2 eps 2^64
    win = np.array([(-(mu64 + hi64 + 1)) % M64,
                    min(e2 + 2 * mu64 + (hi64 - lo64) + (N + 1) + 4, M64 - 1)], np.uint64)
    bands = []
    for lo, hi in ((mu64, e2 - mu64 - 1), (e2 + mu64, M64 - mu64 - 1)):
        if hi < lo or lo > M64 - 1 or hi < 0:
            lo, hi = M64 - 1, 0
        bands += [max(lo, 0), min(hi, M64 - 1)]
    return win, np.array(bands, np.uint64), mu


def _comb_f(x: np.ndarray, k: int) -> np.ndarray:
    """C(x, k) of a float array of integers x >= 0 (0 where x < k), by the
    product formula; relative error below (2 k + 1) 2^-53."""
    out = np.ones_like(x, dtype=np.float64)
    for i in range(k):
        out = out * np.maximum(x - i, 0.0) / (i + 1)
    return out


def upper_windows_many(U: UpperTable, Ns, taus, delta: int, W: int):
    """upper_windows for many (N, tau) pairs at once (numpy, binary64 with
    the same outward margins): windows uint64 (n, 2), thresholds uint64
    (n, 4).  The largest N sets the common offset range X of U's derivative
    bounds, which only widens the others' bounds."""
    d = delta
    if not 1 <= d <= min(U.Du, 8):
        raise ValueError("degree must be between 1 and the upper degree")
    Ns = np.asarray(Ns, dtype=np.int64)
    taus = np.asarray(taus, dtype=np.int64)
    Nf, Tf = Ns.astype(np.float64), taus.astype(np.float64)
    Du = U.Du
    c = [float(x) for x in U.coeffs]
    ca = [abs(x) * _UP for x in c]
    X = float(U.count + d * int(Ns.max()) + d)
    fac = [float(math.factorial(k)) for k in range(Du + 1)]
    Xp = [X ** e * _UP for e in range(Du + 1)]
    Mx = [sum(ca[k] * fac[k] / fac[k - n] * Xp[k - n] for k in range(n, Du + 1)) * _UP
          for n in range(Du + 1)]
    en = [float(U.shift_error(n)) * _UP for n in range(Du + 1)]
    cN = [_comb_f(Nf - 1, j) * _UP for j in range(Du + 1)]
    cT = [_comb_f(Tf - 1, l) * _UP for l in range(Du + 1)]
    drop, keptE = {}, {}
    for j in range(Du + 1):
        for l in range(Du - j + 1):
            if j + l > d:
                drop[(j, l)] = Nf ** l * Mx[j + l] * _UP
            else:
                acc = np.zeros_like(Nf)
                for n in range(j + l, Du + 1):
                    acc = acc + en[n] * 2.0 ** l * _comb_f(l * Nf, n - j) * _UP
                keptE[(j, l)] = acc * _UP
    e_drop = sum(v * cT[l] * cN[j] for (j, l), v in drop.items()) * _UP
    e_shift = sum(v * cT[l] * cN[j] for (j, l), v in keptE.items()) * _UP
    rsum = sum(cN[j] * cT[l] for j in range(d + 1) for l in range(d - j + 1)) * _UP
    e_rw = rsum * 2.0 ** -W * _UP
    mu = (float(U.e_approx) * _UP + e_drop + e_shift + e_rw) * _UP
    t_lo = np.zeros_like(Nf)
    t_hi = np.zeros_like(Nf)
    for j in range(2, d + 1):
        base = c[j] * fac[j]
        lo_j = hi_j = base
        mag = abs(base)
        for k in range(j + 1, Du + 1):
            term = c[k] * fac[k] / fac[k - j] * X ** (k - j)
            lo_j += min(term, 0.0)
            hi_j += max(term, 0.0)
            mag += abs(term)
        slack = (sum((drop[(j, l)] * cT[l] for l in range(d - j + 1, Du - j + 1)),
                     np.zeros_like(Nf))
                 + sum(keptE[(j, l)] * cT[l] for l in range(d - j + 1))
                 + 2.0 ** (-W - 1) * sum(cT[l] for l in range(d - j + 1))) * _UP
        margin = mag * 2.0 ** -40 + slack
        t_lo = t_lo + np.minimum(lo_j - margin, 0.0) * cN[j] * _UP
        t_hi = t_hi + np.maximum(hi_j + margin, 0.0) * cN[j] * _UP
    t_lo = t_lo * _UP
    t_hi = t_hi * _UP
    n = len(Ns)
    win = np.zeros((n, 2), np.uint64)
    thr = np.zeros((n, 4), np.uint64)
    e2 = 1 << (65 - U.s)
    for i in range(n):
        mu64 = math.ceil(float(mu[i]) * 2.0 ** 64)
        hi64 = math.ceil(float(t_hi[i]) * 2.0 ** 64)
        lo64 = math.floor(float(t_lo[i]) * 2.0 ** 64)
        win[i, 0] = (-(mu64 + hi64 + 1)) % M64
        win[i, 1] = min(e2 + 2 * mu64 + (hi64 - lo64) + int(Ns[i]) + 1 + 4, M64 - 1)
        bands = []
        for lo, hi in ((mu64, e2 - mu64 - 1), (e2 + mu64, M64 - mu64 - 1)):
            if hi < lo or lo > M64 - 1 or hi < 0:
                lo, hi = M64 - 1, 0
            bands += [max(lo, 0), min(hi, M64 - 1)]
        thr[i] = bands
    return win, thr
