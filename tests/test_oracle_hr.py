"""Pins for oracle/hr.py: pipeline oracle vs per-argument brute force (Def. 2-3)."""
import math
import random

import mpmath
import pytest
from mpmath import mpf

from oracle import hr
from oracle.search import brute_hits
from oracle.tabulate import piece_ab, straightforward_rows
from oracle.taylor import FUNCTIONS, Job, eps_approx, eps_round, initial_table

STARTS = {"exp": 1.0, "exp2": 1.0, "log": 3.0, "sin": 1.0, "cos": 1.0}


@pytest.mark.parametrize("fname", FUNCTIONS)
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_pipeline_equals_bruteforce(fname, mode):
    """P1: the three-phase oracle and per-argument evaluation agree on a small
    range with a loose eps (so that there are many HR cases)."""
    X0 = STARTS[fname] + (0.37 if fname == "log" else 0.0)
    job = Job(fname, X0, 1 << 13, 8, mode, 1 << 6, 1 << 4, 3, 128)
    bf = hr.hr_bruteforce(job)
    assert len(bf) > 20
    assert hr.pipeline(job) == bf
    assert hr.pipeline(job, use_filter=False) == bf


def test_pipeline_equals_bruteforce_wider_words():
    job = Job("exp", 1.25, 1 << 14, 9, "rn", 1 << 7, 1 << 4, 4, 256)
    assert hr.pipeline(job) == hr.hr_bruteforce(job)


def test_hr_count_is_poisson_like():
    """P2: the number of HR cases is about 2 eps * #args."""
    job = Job("exp", 1.0, 1 << 18, 10, "rn", 1 << 10, 1 << 6, 3, 128)
    n = len(hr.pipeline(job))
    expect = 2 * 2 ** -10 * job.count
    assert abs(n - expect) < 5 * expect ** 0.5


def test_piece_window_contains_every_hr_argument():
    """Every HR argument of a piece lies in the widened degree-1 window."""
    job = Job("exp2", 1.0, 1 << 13, 7, "rn", 1 << 6, 1 << 4, 3, 128)
    cases = set(hr.hr_bruteforce(job))
    assert len(cases) > 50
    with mpmath.workprec(128):
        for t in range(job.n_sub):
            T = initial_table(job, t)
            mu = eps_approx(job, t) + eps_round(job)
            for i in range(job.tau):
                rows = straightforward_rows(T, job.delta, i, job.W)
                a, b = piece_ab(rows, job.W)
                LO, D = hr.piece_window(rows, job, mu)
                window = set(brute_hits(a, b, job.N, D, lo=LO))
                base = t * job.per_sub + i * job.N
                for m in cases:
                    if base <= m < base + job.N:
                        assert m - base in window


def _float_rounding_is_hr(fname, X0, m, s, mode):
    """Def. 2-3 restated through binary64 rounding done by the libraries:
    with u = ulp(f(X)) (math.ulp of the rounded value; the slices stay
    inside one binade) and the interval (f(X) - eps u, f(X) + eps u),
    X is a round-to-nearest case iff its two ends round to nearest to
    different binary64 numbers (a midpoint lies between them), and a
    directed case iff rounding the upper end down lands above the lower
    end (a binary64 number lies between them)."""
    X = X0 + m * math.ulp(X0)                 # exact: the argument grid
    with mpmath.workprec(320):
        y = {"exp": mpmath.exp, "exp2": lambda t: mpmath.power(2, t), "log": mpmath.log,
             "sin": mpmath.sin, "cos": mpmath.cos}[fname](mpf(X))
        u = mpf(math.ulp(float(y)))
        lo, hi = y - mpf(2) ** -s * u, y + mpf(2) ** -s * u
        if mode == "rn":
            return float(lo) != float(hi)
        return mpf(hi, prec=53, rounding="f") > lo


@pytest.mark.parametrize("fname", FUNCTIONS)
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_hr_test_equals_binary64_rounding(fname, mode):
    """The oracle's HR decision (distance of f(X)/u_f - c to the integers,
    c = 1/2 for nearest, 0 for directed) equals the rounding restatement on
    random arguments with eps = 2^-3, where about a quarter of them are
    cases.  A swapped c, a wrong ulp or a window of eps instead of 2 eps
    fails it."""
    rng = random.Random(hash((fname, mode)) & 0xffff)
    X0 = STARTS[fname] + (0.37 if fname == "log" else 0.0)
    job = Job(fname, X0, 1 << 40, 3, mode, 1, 1 << 40, 1, 128)
    hits = 0
    for _ in range(300):
        m = rng.randrange(1 << 40)
        got = hr.decide(job, m)
        assert got == _float_rounding_is_hr(fname, X0, m, 3, mode), m
        hits += got
    assert 40 < hits < 120


@pytest.mark.parametrize("X0", [1.0, 2.0])
def test_exact_power_of_two_is_directed_never_nearest(X0):
    """2^x at x = 1 and x = 2 is exactly 2 and 4: at distance 0 from a
    binary64 number, so a directed HR case at every eps, and half an ulp
    from the nearest midpoint, never a round-to-nearest one (Def. 2-3).
    Checked through the per-argument test, the per-argument brute force and
    the three-phase pipeline, at a loose eps (many other cases) and a tight
    one (it is then the only case of the range)."""
    for s in (6, 40):
        for mode in ("dir", "rn"):
            job = Job("exp2", X0, 1 << 12, s, mode, 1 << 6, 1 << 6, 3, 128)
            want = mode == "dir"
            assert hr.decide(job, 0) is want
            assert (0 in hr.pipeline(job)) is want
            if s == 6:
                assert (0 in hr.hr_bruteforce(job)) is want
            else:
                assert hr.pipeline(job) == ([0] if want else [])
