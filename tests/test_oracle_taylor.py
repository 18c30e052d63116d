"""Pins for oracle/taylor.py (Sec. 3.1 change of variable, Sec. 5.1 tables)."""
import random
from math import comb

import mpmath
import pytest
from mpmath import mpf

from oracle.tabulate import evaluate, straightforward_rows
from oracle.taylor import (FUNCTIONS, Job, arg_ulp, derivative, eps_approx,
                           eps_round, exact_table, f_value, initial_table,
                           out_ulp, sub_start, taylor_coeffs)

STARTS = {"exp": 1.0, "exp2": 1.0, "log": 3.0, "sin": 1.0, "cos": 1.0}


@pytest.mark.parametrize("fname", FUNCTIONS)
def test_derivatives_match_numerical_differentiation(fname):
    with mpmath.workprec(200):
        X = mpf("1.2345")
        f = {"exp": mpmath.exp, "exp2": lambda x: mpmath.power(2, x), "log": mpmath.log,
             "sin": mpmath.sin, "cos": mpmath.cos}[fname]
        for n in range(6):
            num = mpmath.diff(f, X, n)
            assert abs(num - derivative(fname, X, n)) < mpf(2) ** -100 * (1 + abs(num))


def test_ulps():
    assert arg_ulp(1.0) == mpf(2) ** -52
    assert arg_ulp(1.9999) == mpf(2) ** -52
    assert arg_ulp(3.0) == mpf(2) ** -51
    assert out_ulp(Job("exp", 1.0, 1 << 20, 24, "rn", 1 << 8, 1 << 4, 3, 128)) == mpf(2) ** -51
    assert out_ulp(Job("sin", 1.0, 1 << 20, 24, "rn", 1 << 8, 1 << 4, 3, 128)) == mpf(2) ** -53
    assert out_ulp(Job("log", 3.0, 1 << 20, 24, "rn", 1 << 8, 1 << 4, 3, 128)) == mpf(2) ** -52
    with pytest.raises(ValueError):      # exp crosses 4 near X = ln 4
        out_ulp(Job("exp", 1.386, 1 << 50, 24, "rn", 1 << 8, 1 << 4, 3, 128))


def _g(job, t, x, prec):
    """g(x) = f(X_t + x h)/u_f - c + eps, directly from f."""
    with mpmath.workprec(prec):
        X = sub_start(job, t) + x * arg_ulp(job.X0)
        c = mpf(1) / 2 if job.mode == "rn" else 0
        return f_value(job.fname, X) / out_ulp(job) - c + mpf(2) ** (-job.s)


@pytest.mark.parametrize("fname", FUNCTIONS)
def test_taylor_within_lagrange_bound(fname):
    """|R_t(x) - g(x)| <= eps_approx on the whole sub-interval, and the
    bound is not vacuous (the error at the far end reaches a fair part of it)."""
    job = Job(fname, STARTS[fname], 1 << 24, 24, "rn", 1 << 10, 1 << 6, 3, 192)
    t = 5
    with mpmath.workprec(400):
        c = taylor_coeffs(job, t, 400)
        ea = eps_approx(job, t)
        worst = mpf(0)
        for x in [0, 1, 17, 1000, job.per_sub // 2, job.per_sub - 1]:
            R = sum(cn * mpf(x) ** n for n, cn in enumerate(c))
            err = abs(R - _g(job, t, x, 400))
            assert err <= ea
            worst = max(worst, err)
        if fname in ("exp", "exp2", "log"):      # derivative of constant sign
            assert worst > ea / 4


def test_exp_table_matches_closed_form():
    """For f = exp the hierarchical table has a closed form:
    Delta_N^l Delta_1^j g(0) = e^{X_t} (e^h - 1)^j (e^{N h} - 1)^l / u_f for
    j + l >= 1.  The Taylor-based table must agree within the propagated
    approximation error 2^(j+l) eps_approx (catches swapped j and l)."""
    job = Job("exp", 1.0, 1 << 22, 20, "rn", 1 << 9, 1 << 5, 4, 256)
    t = 3
    with mpmath.workprec(512):
        T = exact_table(job, t, 512)
        h = arg_ulp(job.X0)
        uf = out_ulp(job)
        Xt = sub_start(job, t)
        ea = eps_approx(job, t)
        for j in range(job.delta + 1):
            for l in range(job.delta - j + 1):
                if j + l == 0:
                    continue
                closed = mpmath.exp(Xt) * (mpmath.exp(h) - 1) ** j * (mpmath.exp(job.N * h) - 1) ** l / uf
                assert abs(T[j][l] - closed) <= 2 ** (j + l) * ea, (j, l)


@pytest.mark.parametrize("fname", FUNCTIONS)
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_rounded_table_reproduces_g(fname, mode):
    """Piece values from the rounded W-bit table equal g(i N + x) mod 1 within
    eps_approx + eps_round (Sec. 5: the table plus shifts is the whole
    polynomial generation step)."""
    job = Job(fname, STARTS[fname], 1 << 24, 24, mode, 1 << 9, 1 << 5, 3, 128)
    rng = random.Random(len(fname))
    for t in (0, 7):
        T = initial_table(job, t)
        mu = eps_approx(job, t) + eps_round(job)
        for _ in range(12):
            i, x = rng.randrange(job.tau), rng.randrange(job.N)
            V = evaluate(straightforward_rows(T, job.delta, i, job.W), x, job.W)
            with mpmath.workprec(300):
                g = _g(job, t, i * job.N + x, 300)
                diff = mpf(V) / mpf(2) ** job.W - (g - mpmath.floor(g))
                diff -= mpmath.nint(diff)
                assert abs(diff) <= mu


ROUND_SHAPES = [(1 << 16, 1 << 3, 3, 128), (2, 1 << 20, 3, 128), (1 << 9, 1 << 9, 4, 128),
                (1 << 12, 1 << 6, 2, 192), (3, 5, 6, 256)]


def _adversarial_rounding_error(N, tau, delta, W):
    """Exact values of a random table placed exactly halfway between two
    W-bit words, every entry rounded up (the worst a rounding to nearest
    can do, all errors of one sign): the change of the value of the last
    piece at its last argument, in units of 2^-(W+1), by the oracle's
    straightforward shift and piece evaluation."""
    rng = random.Random(N * 1000003 + tau)
    half = [[2 * rng.randrange(1 << W) + 1 for _ in range(delta - j + 1)]
            for j in range(delta + 1)]                      # units of 2^-(W+1)
    up = [[((v + 1) // 2) % (1 << W) for v in row] for row in half]
    i, x = tau - 1, N - 1
    V = evaluate(straightforward_rows(up, delta, i, W), x, W)
    exact = sum(half[j][l] * comb(i, l) * comb(x, j)
                for j in range(delta + 1) for l in range(delta - j + 1))
    err = (2 * V - exact) % (1 << (W + 1))
    return err if err < 1 << W else err - (1 << (W + 1))


@pytest.mark.parametrize("N,tau,delta,W", ROUND_SHAPES)
def test_eps_round_reached_by_adversarial_rounding(N, tau, delta, W):
    """eps_round bounds the worst rounding of a table and is reached within
    its stated factor 2: the adversarial table of _adversarial_rounding_error
    moves the value by exactly half of it.  Shapes with N >> tau and with
    tau >> N make a bound without the C(N-1, j) or without the C(tau-1, l)
    factor fail, and a product of the two full sums (instead of the
    triangle j + l <= delta) is loose by far more than 4."""
    err = _adversarial_rounding_error(N, tau, delta, W)
    bound = eps_round(Job("exp", 1.0, N * tau, 20, "rn", N, tau, delta, W)) * mpf(2) ** (W + 1)
    assert 0 < err <= bound
    assert 4 * err >= bound


@pytest.mark.parametrize("N,tau,delta,W", ROUND_SHAPES)
def test_product_round_bound_reached_by_adversarial_rounding(N, tau, delta, W):
    """The same pin for the device path's own bound (prep.round_bound),
    which sets its windows and thresholds and the autotuner's width."""
    from paper_1211_3056_amd.prep import round_bound
    err = _adversarial_rounding_error(N, tau, delta, W)
    bound = round_bound(N, tau, delta, W) * mpf(2) ** (W + 1)
    assert 0 < err <= bound
    assert 4 * err >= bound


def test_eps_round_small_against_eps_approx():
    job = Job("exp", 1.0, 1 << 24, 24, "rn", 1 << 9, 1 << 5, 3, 128)
    assert eps_round(job) < mpf(2) ** -90
    assert eps_approx(job, 0) < mpf(2) ** -40
