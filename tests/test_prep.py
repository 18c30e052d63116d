"""CPU checks of the product's host preparation and planning (no GPU):
tables equal the oracle's independently computed tables, every HR argument
lies in the product's degree-1 window, the recheck thresholds never
contradict per-argument brute force, and the autotuner's choices are sound."""
import math

import numpy as np
import pytest

import synth
from oracle import hr as ohr
from oracle.search import brute_hits
from oracle.tabulate import evaluate, piece_ab, straightforward_rows, top64
from oracle.taylor import Job, initial_table
from paper_1211_3056_amd import autotune
from paper_1211_3056_amd.plan import BatchJob, plan_job
from paper_1211_3056_amd.prep import JobSpec, SubPreparer, output_ulp_range, prepare

STARTS = {"exp": 1.0, "exp2": 1.0, "log": 3.37, "sin": 1.0, "cos": 1.0}


def _ints(table, W):
    L = W // 64
    return [sum(int(table[e, l]) << (64 * l) for l in range(L)) for e in range(table.shape[0])]


def _rows_T(flat, d):
    T, pos = [], 0
    for j in range(d + 1):
        T.append(flat[pos:pos + d - j + 1])
        pos += d - j + 1
    return T


@pytest.mark.parametrize("fname", ["exp", "exp2", "log", "sin", "cos"])
@pytest.mark.parametrize("W,delta,N,tau", [(128, 3, 1 << 6, 1 << 4), (256, 4, 1 << 9, 1 << 5)])
def test_tables_equal_oracle(fname, W, delta, N, tau):
    spec = JobSpec(fname, STARTS[fname], N * tau * 4, 20, "rn", N, tau, delta, W)
    P = prepare(spec)
    job = Job(fname, STARTS[fname], N * tau * 4, 20, "rn", N, tau, delta, W)
    for r, t in enumerate(P.subs):
        flat = [v for row in initial_table(job, int(t)) for v in row]
        assert _ints(P.tables[r], W) == flat


@pytest.mark.parametrize("fname", ["exp", "exp2", "log", "sin", "cos"])
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_windows_and_thresholds_against_bruteforce(fname, mode):
    """Every HR argument of each piece is a candidate of the product's
    window; every value the thresholds call certain agrees with brute force."""
    N, tau, d, W = 1 << 6, 1 << 4, 3, 128
    spec = JobSpec(fname, STARTS[fname], N * tau * 8, 8, mode, N, tau, d, W)
    job = Job(fname, STARTS[fname], N * tau * 8, 8, mode, N, tau, d, W)
    cases = set(ohr.hr_bruteforce(job))
    assert len(cases) > 20
    P = prepare(spec)
    n_cand = 0
    for r, t in enumerate(P.subs):
        T = _rows_T(_ints(P.tables[r], W), d)
        lo, width = int(P.win[r, 0]), int(P.win[r, 1])
        hr_lo, hr_hi, rej_lo, rej_hi = (int(x) for x in P.thr[r])
        for i in range(tau):
            rows = straightforward_rows(T, d, i, W)
            a, b = piece_ab(rows, W)
            cand = set(brute_hits(a, b, N, width, lo=lo))
            n_cand += len(cand)
            base = int(t) * spec.per_sub + i * N
            for x in range(N):
                m = base + x
                tv = top64(evaluate(rows, x, W), W)
                if m in cases:
                    assert x in cand
                    assert not (rej_lo <= tv <= rej_hi)
                elif hr_lo <= tv <= hr_hi:
                    pytest.fail(f"value certain HR but brute force says no: {m}")
    assert n_cand < spec.count          # the window actually filters


def test_partial_subintervals_prepare_like_whole_ones():
    """A sub-interval cut short keeps the table of its start; only the error
    budget (length, tau) changes."""
    uf = output_ulp_range("exp", 1.0, 1 << 20)
    sp = SubPreparer("exp", 1.0, 20, "rn", 3, 128, uf)
    t_full, w_full, _ = sp.prepare(1 << 16, 1 << 16, 1000)
    t_part, w_part, _ = sp.prepare(1 << 16, 12345, 1000)
    assert np.array_equal(t_full, t_part)
    assert int(w_part[1]) <= int(w_full[1])


def test_autotuner_choices():
    uf = output_ulp_range("exp", 1.0, 1 << 40)
    # degree: the 2^28-argument sub-intervals of the batch workload need 3
    assert autotune.choose_degree("exp", 1.0, 1 << 28, 28, uf) == 3
    assert autotune.choose_degree("exp", 1.0, 1 << 20, 28, uf) <= 2
    # width grows with the table-rounding amplification
    assert autotune.choose_width([(1 << 12, 1 << 16)], 3, 28) == 128
    assert autotune.choose_width([(1 << 20, 1 << 16)], 4, 32) == 128
    assert autotune.choose_width([(1 << 20, 1 << 16)], 6, 32) >= 192
    # piece length: tighter thresholds favour shorter pieces
    assert autotune.choose_N("exp", 1.0, 1 << 36, 28, uf) <= autotune.choose_N("exp", 1.0, 1 << 36, 20, uf)
    # item split covers every piece exactly once, 64 lanes x nu each
    items = autotune.split_sub(1000, 1 << 12, 5000.0, 50.0)
    assert sum(n for _, n, _ in items) == 1000
    assert all(n <= 64 * nu for _, n, nu in items)
    assert [p for p, _, _ in items] == sorted(p for p, _, _ in items)


def test_plan_job_ragged_ranges():
    pj = plan_job(BatchJob("sin", 1.25, 300_001, 11, "rn", sub_len=65_536, N=[1000, 777, 4096, 333, 5000]))
    assert [s.length for s in pj.subs] == [65536] * 4 + [300_001 - 4 * 65536]
    assert sum(s.length for s in pj.subs) == 300_001
    assert pj.subs[-1].pieces == math.ceil(pj.subs[-1].length / 5000)
    with pytest.raises(ValueError):
        plan_job(BatchJob("exp", 1.3862943, 1 << 40, 20, "rn"))      # crosses 4


def test_workload_generators_are_seeded():
    a, b = synth.config4(), synth.config4()
    assert a == b and len(a) == 16
    c5 = synth.config5(n_jobs=50)
    assert c5 == synth.config5(n_jobs=50)
    for d in c5:
        output_ulp_range(d["fname"], d["X0"], d["count"])     # one output binade each


def test_prepare_with_pool_equals_serial():
    """Sub-intervals prepared in chunks by worker processes give the same
    tables, windows and thresholds as the serial loop."""
    from paper_1211_3056_amd import serve
    spec = JobSpec("exp", 1.0, 1 << 26, 24, "rn", 1 << 12, 1 << 8, 3, 192)
    pool = serve.make_pool(2)
    try:
        a, b = prepare(spec), prepare(spec, pool=pool)
    finally:
        pool.shutdown()
    assert spec.n_sub >= 4
    for f in ("tables", "win", "thr", "subs"):
        assert np.array_equal(getattr(a, f), getattr(b, f))


def test_error_budget_above_eps_gives_empty_hr_band():
    """A degree too small for eps (degree 1 over 2^24 arguments of exp with
    eps = 2^-8: the Lagrange remainder alone exceeds 2 eps) leaves no value
    that can be certified HR: the HR band is empty (lo > hi) instead of
    negative, and the reject band still holds the values far from every
    breakpoint."""
    uf = output_ulp_range("exp", 1.0, 1 << 24)
    sp = SubPreparer("exp", 1.0, 8, "rn", 1, 128, uf)
    _, win, thr = sp.prepare(0, 1 << 24, 1 << 12)
    hr_lo, hr_hi, rej_lo, rej_hi = (int(x) for x in thr)
    assert hr_lo == 2 ** 64 - 1 and hr_hi == 0
    assert 0 < rej_lo < rej_hi < 2 ** 64
    assert int(win[1]) > 2 ** 58          # the window covers the whole budget


def test_value_bands_closed_forms():
    from mpmath import mpf

    from paper_1211_3056_amd.prep import value_bands
    eps = mpf(2) ** -20
    assert value_bands(mpf(0), eps) == [0, 2 ** 45 - 1, 2 ** 45, 2 ** 64 - 1]
    # mu = 2^-30: HR band [2^34, 2^45 - 2^34 - 1], reject [2^45 + 2^34, 2^64 - 2^34 - 1]
    mu = mpf(2) ** -30
    assert value_bands(mu, eps) == [2 ** 34, 2 ** 45 - 2 ** 34 - 1, 2 ** 45 + 2 ** 34,
                                    2 ** 64 - 2 ** 34 - 1]
    assert value_bands(mpf(2) ** -19, eps)[:2] == [2 ** 64 - 1, 0]
    assert value_bands(mpf(1) / 2, eps) == [2 ** 64 - 1, 0, 2 ** 64 - 1, 0]


# ---------------------------------------------------------------- upper level

@pytest.mark.parametrize("fname", ["exp", "exp2", "log", "sin", "cos"])
@pytest.mark.parametrize("count,S,Du,Wu", [(1 << 36, 1 << 24, 6, 320), (1 << 20, 1 << 10, 4, 192)])
def test_upper_table_equals_oracle(fname, count, S, Du, Wu):
    """The product's upper table (fixed-point monomials through exact
    integer matrices) equals the oracle's (Newton interpolation of mpmath
    values on the grid, Sec. 5.1), word for word."""
    from oracle.taylor import upper_table as oracle_upper
    from paper_1211_3056_amd.prep import upper_table
    U = upper_table(fname, STARTS[fname], count, 20, "rn", S, Du, Wu)
    ref = oracle_upper(fname, STARTS[fname], count, 20, "rn", Du, S, Wu)
    assert _ints(U.words, Wu) == [v for row in ref for v in row]


@pytest.mark.parametrize("fname", ["exp", "exp2", "log", "sin", "cos"])
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_upper_windows_against_bruteforce(fname, mode):
    """Sub-interval tables made from the upper table (by the oracle's
    two-level shift, standing in for the device): every HR argument of each
    piece is a candidate of the window upper_windows gives, and no value the
    thresholds call certainly HR (or certainly not) contradicts the
    per-argument brute force."""
    from oracle.tabulate import subinterval_table
    from paper_1211_3056_amd.prep import upper_table, upper_windows
    N, tau, d, W, Du, Wu, T = 1 << 6, 1 << 4, 3, 128, 5, 192, 8
    S = N * tau
    count = S * T
    job = Job(fname, STARTS[fname], count, 8, mode, N, tau, d, W)
    cases = set(ohr.hr_bruteforce(job))
    assert len(cases) > 20
    U = upper_table(fname, STARTS[fname], count, 8, mode, S, Du, Wu)
    win, thr, mu = upper_windows(U, N, tau, d, W)
    assert mu < 2.0 ** -40
    lo, width = int(win[0]), int(win[1])
    hr_lo, hr_hi, rej_lo, rej_hi = (int(x) for x in thr)
    Uw = _ints(U.words, Wu)
    Urows = _rows_T(Uw, Du)
    n_cand = 0
    for t in range(T):
        Tt = subinterval_table(Urows, Du, t, N, d, Wu, W)
        for i in range(tau):
            rows = straightforward_rows(Tt, d, i, W)
            a, b = piece_ab(rows, W)
            cand = set(brute_hits(a, b, N, width, lo=lo))
            n_cand += len(cand)
            base = t * S + i * N
            for x in range(N):
                m = base + x
                tv = top64(evaluate(rows, x, W), W)
                if m in cases:
                    assert x in cand, m
                    assert not (rej_lo <= tv <= rej_hi), m
                elif hr_lo <= tv <= hr_hi:
                    pytest.fail(f"value certain HR but brute force says no: {m}")
    assert n_cand < count


def test_upper_error_budget_shapes():
    """At the large workload's shape (exp, 2^40 arguments, sub-intervals of
    2^28, pieces of 2^18, degree 4 at 256 bits) a degree-7 upper polynomial
    at 320 bits leaves an error below eps 2^-24 and a window within 0.1% of
    the per-sub-interval Taylor windows; degree 6 is not enough for 2^-12."""
    import mpmath
    from paper_1211_3056_amd.prep import upper_table, upper_windows
    U7 = upper_table("exp", 1.0, 1 << 40, 32, "rn", 1 << 28, 7, 320)
    win, thr, mu = upper_windows(U7, 1 << 18, 1 << 10, 4, 256)
    assert mu < mpmath.mpf(2) ** (-32 - 24)
    P = prepare(JobSpec(**synth.CONFIG3), subs=[0, 4095])
    assert int(P.win[:, 1].max()) <= int(win[1]) < int(P.win[:, 1].max()) * 1.001
    U6 = upper_table("exp", 1.0, 1 << 40, 32, "rn", 1 << 28, 6, 320)
    assert U6.e_approx > mpmath.mpf(2) ** (-32 - 12)


@pytest.mark.parametrize("fname,X0,count,S,Du,Wu,N,tau,d,W,s", [
    ("exp", 1.0, 1 << 40, 1 << 28, 7, 320, 1 << 18, 1 << 10, 4, 256, 32),
    ("exp", 1.0, 1 << 32, 1 << 24, 4, 256, 1 << 16, 1 << 8, 3, 192, 24),
    ("log", 3.0, 1 << 36, 1 << 28, 6, 320, 5000, 53688, 3, 128, 28),
    ("sin", 1.0, 1 << 34, 1 << 26, 6, 256, 1 << 14, 1 << 12, 3, 128, 20),
    ("exp2", 1.25, 1 << 30, 1 << 20, 5, 192, 1 << 10, 1 << 10, 2, 128, 28)])
def test_float_windows_contain_precise_ones(fname, X0, count, S, Du, Wu, N, tau, d, W, s):
    """The binary64 bounds of upper_windows contain the 192-bit ones: the
    window starts at or before the precise start and ends at or after its
    end, and each certainty band lies inside the precise band."""
    from paper_1211_3056_amd.prep import upper_table, upper_windows, upper_windows_precise
    U = upper_table(fname, X0, count, s, "rn", S, Du, Wu)
    wf, tf, muf = upper_windows(U, N, tau, d, W)
    wp, tp, mup = upper_windows_precise(U, N, tau, d, W)
    shift = (int(wp[0]) - int(wf[0])) % (1 << 64)
    assert shift < 1 << 16
    assert int(wf[1]) >= int(wp[1]) + shift
    assert muf >= float(mup)
    for b in (0, 2):
        lo_f, hi_f, lo_p, hi_p = int(tf[b]), int(tf[b + 1]), int(tp[b]), int(tp[b + 1])
        if lo_f <= hi_f:
            assert lo_p <= lo_f and hi_f <= hi_p


def test_vectorised_windows_contain_precise_ones():
    """upper_windows_many over uneven piece lengths (the batched workload's
    shapes) contains the 192-bit bounds of every (N, tau) pair."""
    from paper_1211_3056_amd.prep import upper_table, upper_windows_many, upper_windows_precise
    U = upper_table("exp", 1.0, 1 << 34, 28, "rn", 1 << 28, 6, 320)
    rng = synth.rng(9)
    Ns = rng.integers(1 << 12, (1 << 20) + 1, 12)
    Ns[0], Ns[1] = 1 << 12, 1 << 20
    taus = -(-(1 << 28) // Ns)
    taus[2] = 1
    win, thr = upper_windows_many(U, Ns, taus, 3, 128)
    for i in range(len(Ns)):
        wp, tp, _ = upper_windows_precise(U, int(Ns[i]), int(taus[i]), 3, 128)
        # the common offset range (largest N) may start the window earlier
        shift = (int(wp[0]) - int(win[i, 0])) % (1 << 64)
        assert shift < int(wp[1]) // 64 and int(win[i, 1]) >= int(wp[1]) + shift, i
        for b in (0, 2):
            if int(thr[i, b]) <= int(thr[i, b + 1]):
                assert int(tp[b]) <= int(thr[i, b]) and int(thr[i, b + 1]) <= int(tp[b + 1])


def test_upper_width_choice():
    """The narrowest width the autotuner takes for the large workload (256
    bits at degree 7) adds less than eps 2^-24 to the error budget over 320
    bits, and keeps the device's integer steps exact."""
    from paper_1211_3056_amd.prep import upper_table, upper_windows_precise
    Wu = autotune.choose_upper_width(7, 4096, 1 << 18, 1 << 10, 4, 32)
    assert Wu == 256
    assert (4 * (1 << 18)) ** 7 < 1 << Wu
    mus = []
    for w in (Wu, 320):
        U = upper_table("exp", 1.0, 1 << 40, 32, "rn", 1 << 28, 7, w)
        mus.append(upper_windows_precise(U, 1 << 18, 1 << 10, 4, 256)[2])
    assert mus[0] - mus[1] < 2.0 ** (-32 - 24)
    # a width too narrow for the shape is refused
    with pytest.raises(ValueError):
        autotune.choose_upper_width(10, 1 << 20, (1 << 32) - 1, 1 << 20, 8, 40)
