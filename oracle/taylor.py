"""Taylor polynomials, hierarchical initial tables and error bounds (oracle).

Sec. 3.1 (definitions, change of variable) and Sec. 5.1 (hierarchical method,
Newton interpolation in the binomial basis, Fig. 6) of the paper.

Scaled problem.  For binary64 arguments X = X_t + x h (h = ulp of X, constant
inside a binade; x an integer, the change of variable of Sec. 3.1) and
f(X) inside one output binade with ulp u_f, an argument is a (53, eps) HR case
when the scaled value y = f(X)/u_f is within eps of a rounding breakpoint
(Def. 2-3).  Round-to-nearest breakpoints are the midpoints y in Z + 1/2,
directed ones the integers.  With c = 1/2 (nearest) or c = 0 (directed) the
test of Sec. 3.1 reads

    {y - c + eps} < 2 eps.

R_t(x) is the degree-delta Taylor polynomial of g(x) = f(X_t + x h)/u_f - c +
eps at x = 0 (coefficients f^(n)(X_t) h^n / (n! u_f)); the HR search runs on
R_t's pieces.  Derivatives use their closed forms (exp: e^X, 2^x: ln2^n 2^X,
log: (-1)^(n-1) (n-1)!/X^n, sin and cos: phase shifts by n pi/2), evaluated by
mpmath at W + 256 bits.

The initial table of sub-interval t follows the hierarchical method: values
R_t(s N + m) on a (delta+1) x (delta+1) grid, forward differences in m give
r_j(s) = Delta^j[R_t](s N) (Newton interpolation, Fig. 6), forward
differences in s give T[j][l] = Delta_s^l r_j(0).  Each entry is then rounded
once to the nearest W-bit fraction mod 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from math import comb

import mpmath
from mpmath import mpf

FUNCTIONS = ("exp", "exp2", "log", "sin", "cos")


@dataclass(frozen=True)
class Job:
    """One HR search job: f over `count` consecutive binary64 arguments.

    The range [X0, X0 + count h) is cut into sub-intervals of tau * N
    arguments, each sub-interval into tau pieces of N arguments (Sec. 5).
    eps = 2^-s in units of the output ulp.
    """

    fname: str
    X0: float
    count: int
    s: int
    mode: str       # "rn" (nearest) or "dir" (directed)
    N: int
    tau: int
    delta: int
    W: int

    @property
    def per_sub(self) -> int:
        return self.tau * self.N

    @property
    def n_sub(self) -> int:
        if self.count % self.per_sub:
            raise ValueError("count must be a multiple of tau * N")
        return self.count // self.per_sub


def arg_ulp(X: float) -> mpf:
    """ulp of a binary64 X > 0: 2^(e - 53) with X = m 2^e, m in [1/2, 1)."""
    _, e = math.frexp(X)
    return mpf(2) ** (e - 53)


def f_value(fname: str, X):
    return {"exp": mpmath.exp, "exp2": lambda x: mpmath.power(2, x),
            "log": mpmath.log, "sin": mpmath.sin, "cos": mpmath.cos}[fname](X)


def derivative(fname: str, X, n: int):
    """f^(n)(X) from its closed form, at the current mpmath precision."""
    X = mpf(X)
    if fname == "exp":
        return mpmath.exp(X)
    if fname == "exp2":
        return mpmath.log(2) ** n * mpmath.power(2, X)
    if fname == "log":
        if n == 0:
            return mpmath.log(X)
        return (-1) ** (n - 1) * mpmath.factorial(n - 1) / X ** n
    if fname == "sin":
        return mpmath.sin(X + n * mpmath.pi / 2)
    if fname == "cos":
        return mpmath.cos(X + n * mpmath.pi / 2)
    raise ValueError(fname)


def out_ulp(job: Job, prec: int = 128) -> mpf:
    """ulp of f over the job's range; the range must stay in one binade.

    All five functions are monotone on the slices used here, so checking the
    two end values is enough.
    """
    with mpmath.workprec(prec):
        h = arg_ulp(job.X0)
        lo = f_value(job.fname, mpf(job.X0))
        hi = f_value(job.fname, mpf(job.X0) + (job.count - 1) * h)
        _, e1 = mpmath.frexp(lo)
        _, e2 = mpmath.frexp(hi)
        if e1 != e2:
            raise ValueError("f changes binade inside the job range")
        return mpf(2) ** (e1 - 53)


def sub_start(job: Job, t: int) -> mpf:
    """X_t, first argument of sub-interval t (exact)."""
    return mpf(job.X0) + t * job.per_sub * arg_ulp(job.X0)


def taylor_coeffs(job: Job, t: int, prec: int):
    """c_n = f^(n)(X_t) h^n / (n! u_f) for n <= delta, with -c + eps added to c_0."""
    with mpmath.workprec(prec):
        h = arg_ulp(job.X0)
        uf = out_ulp(job)
        Xt = sub_start(job, t)
        c = [derivative(job.fname, Xt, n) * h ** n / (mpmath.factorial(n) * uf)
             for n in range(job.delta + 1)]
        offset = mpf(2) ** (-job.s) - (mpf(1) / 2 if job.mode == "rn" else 0)
        c[0] += offset
        return c


def _forward_differences(values):
    """Delta^0..Delta^g at the first point, by iterated subtraction (Fig. 6)."""
    out = []
    cur = list(values)
    while cur:
        out.append(cur[0])
        cur = [cur[m + 1] - cur[m] for m in range(len(cur) - 1)]
    return out


def hierarchical_table(R, delta: int, N: int):
    """T[j][l] = Delta_N^l Delta_1^j R(0) for any callable R (Sec. 5.1).

    r_j(s) = Delta^j[R](s N) comes from Newton interpolation on the grid line
    s N + m (Fig. 6); the table holds the forward differences of r_j in s.
    Works on Python ints (exact) as well as mpf.
    """
    r = [_forward_differences([R(s * N + m) for m in range(delta + 1)])
         for s in range(delta + 1)]
    return [_forward_differences([r[s][j] for s in range(delta - j + 1)])
            for j in range(delta + 1)]


def exact_table(job: Job, t: int, prec: int | None = None):
    """Unrounded T[j][l] = Delta_N^l Delta_1^j R_t(0) as mpf (Sec. 5.1)."""
    d = job.delta
    prec = prec or job.W + 256
    with mpmath.workprec(prec):
        c = taylor_coeffs(job, t, prec)

        def R(x):
            x = mpf(x)
            return sum(c[n] * x ** n for n in range(d + 1))

        return hierarchical_table(R, d, job.N)


def round_word(x, W: int) -> int:
    """Nearest W-bit fraction of {x}, as an integer mod 2^W."""
    return int(mpmath.nint(x * mpf(2) ** W)) % (1 << W)


def initial_table(job: Job, t: int):
    """Rounded initial table of sub-interval t: list of rows T[j][0..delta-j]."""
    T = exact_table(job, t)
    with mpmath.workprec(job.W + 256):
        return [[round_word(v, job.W) for v in row] for row in T]


def eps_approx(job: Job, t: int) -> mpf:
    """Upper bound on |R_t(x) - g(x)| for x in [0, tau N): Lagrange remainder.

    max |f^(delta+1)| over the sub-interval, from closed forms: exp and 2^x
    are increasing (value at the right end), |log^(n)| decreases (value at
    the left end), |sin^(n)|, |cos^(n)| <= 1.
    """
    d = job.delta
    with mpmath.workprec(128):
        h = arg_ulp(job.X0)
        uf = out_ulp(job)
        Xt = sub_start(job, t)
        Xe = Xt + job.per_sub * h
        n = d + 1
        if job.fname == "exp":
            fmax = mpmath.exp(Xe)
        elif job.fname == "exp2":
            fmax = mpmath.log(2) ** n * mpmath.power(2, Xe)
        elif job.fname == "log":
            fmax = mpmath.factorial(n - 1) / Xt ** n
        else:
            fmax = mpf(1)
        bound = fmax * (job.per_sub * h) ** n / (mpmath.factorial(n) * uf)
        return bound * mpf("1.001")


def eps_round(job: Job) -> mpf:
    """Upper bound on the effect of rounding the table entries to W bits.

    Each entry T[j][l] (j + l <= delta, the triangle of Fig. 6) is off by at
    most 2^-(W+1), plus mpmath's error, which is far smaller.  Piece i's
    r_j(i) = sum_l T[j][l] C(i, l) and the piece polynomial at x is
    sum_j r_j(i) C(x, j) (Sec. 5.1-5.2), so the value at (i, x) moves by
    sum_{j+l<=delta} C(x, j) C(i, l) entry errors at most; the binomials
    grow with i and x, so the worst piece and argument are i = tau - 1,
    x = N - 1.  The bound doubles that maximum to cover the half ulp and
    mpmath's error together: 2^-W sum_{j+l<=delta} C(N-1, j) C(tau-1, l).
    """
    d = job.delta
    s = sum(comb(job.N - 1, j) * comb(job.tau - 1, l)
            for j in range(d + 1) for l in range(d - j + 1))
    return mpf(2) ** (-job.W) * s


# ---------------------------------------------------------------- upper level

def upper_coeffs(fname: str, X0: float, count: int, s: int, mode: str, degree: int,
                 prec: int):
    """Monomial coefficients of the upper-level polynomial U of a whole range
    (Sec. 5.1, the top of the hierarchy): the degree-`degree` Taylor
    polynomial of g(x) = f(X0 + x h)/u_f - c + eps at x = 0, with u_f the
    output ulp over the range (which must stay in one binade)."""
    job = Job(fname, X0, count, s, mode, 1, count, degree, 128)
    return taylor_coeffs(job, 0, prec)


def upper_table(fname: str, X0: float, count: int, s: int, mode: str, degree: int,
                S: int, Wu: int):
    """Upper table of a range: U[n][m] = Delta_S^m Delta_1^n U(0) for
    n + m <= degree (the hierarchical table of U with steps 1 and S, Sec.
    5.1 and Fig. 6), each entry rounded once to the nearest Wu-bit fraction.
    Sub-interval t of the range starts at argument t S."""
    prec = Wu + 64 * degree + 512
    with mpmath.workprec(prec):
        c = upper_coeffs(fname, X0, count, s, mode, degree, prec)

        def U(x):
            x = mpf(x)
            return sum(c[k] * x ** k for k in range(degree + 1))

        T = hierarchical_table(U, degree, S)
        return [[round_word(v, Wu) for v in row] for row in T]

