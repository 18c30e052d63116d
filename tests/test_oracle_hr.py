"""Pins for oracle/hr.py: pipeline oracle vs per-argument brute force (Def. 2-3)."""
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


def test_bruteforce_distance_definition():
    """Def. 2-3 on one argument computed by hand: exp(1) in RN mode."""
    job = Job("exp", 1.0, 1, 1, "rn", 1, 1, 1, 128)
    with mpmath.workprec(200):
        y = mpmath.exp(1) / mpf(2) ** -51
        dist = abs((y - mpf(1) / 2) - mpmath.nint(y - mpf(1) / 2))
    assert hr.decide(job, 0) == (dist < mpf(1) / 2)     # eps = 2^-1
    job2 = Job("exp", 1.0, 1, 60, "rn", 1, 1, 1, 128)
    assert hr.decide(job2, 0) is False
