"""The stored full-size oracle HR lists (tests/golden/hr_*.txt, written by
tests/golden/make_lists.py from oracle/ alone) are checked here against the
oracle's exact per-argument test (Def. 2-3, Sec. 3.1): every stored case is
an HR case, and the count is consistent with the density 2 eps of the HR
set (Poisson, except for log whose values move on a lattice)."""
import math

import pytest

import synth
from conftest import golden_hr_lists
from oracle import hr as ohr
from oracle.taylor import Job


def _check_cases(job, cases, sample=None):
    picks = cases if sample is None else cases[:: max(1, len(cases) // sample)]
    for m in picks:
        assert ohr.decide(job, m), m


def test_table3_list():
    got = golden_hr_lists("table3")
    assert got is not None
    cases = got[0]
    n = (1 << 39) + 1
    job = Job("exp", 1.0, n, 32, "dir", 1 << 15, 1 << 13, 3, 192)
    assert len(cases) == len(set(cases)) and all(0 <= m < n for m in cases)
    # 2 eps per argument: 2^39 2^-31 = 256 expected, Poisson spread 16
    assert abs(len(cases) - 256) < 4 * 16
    _check_cases(job, cases)


def test_config3_list():
    got = golden_hr_lists("config3")
    if got is None:
        pytest.skip("hr_config3.txt not generated")
    cases = got[0]
    job = Job(**synth.CONFIG3)
    assert all(0 <= m < job.count for m in cases)
    assert abs(len(cases) - 512) < 4 * math.sqrt(512)
    _check_cases(job, cases, sample=64)


def test_config4_list():
    got = golden_hr_lists("config4")
    if got is None:
        pytest.skip("hr_config4.txt not generated")
    jobs = [d for d in synth.config4() if d["fname"] != "log"]     # log: see make_lists.py
    assert sorted(got) == [d["job_id"] for d in jobs]
    total = expect = 0
    for d in jobs:
        cases = got[d["job_id"]]
        assert all(0 <= m < d["count"] for m in cases)
        job = Job(d["fname"], d["X0"], d["count"], d["s"], d["mode"], 1 << 16, 1 << 12, 3, 128)
        _check_cases(job, cases, sample=4)
        total += len(cases)
        expect += 2 * 2.0 ** -d["s"] * d["count"]
    assert abs(total - expect) < 4 * math.sqrt(expect)


def test_config4_log_list():
    """The log jobs of the batched workload: every sampled case is HR; the
    count is not held to the 2 eps density (near 3 the values of log sit
    close to a lattice mod 1), only to lie within a factor of it."""
    got = golden_hr_lists("config4_log")
    if got is None:
        pytest.skip("hr_config4_log.txt not generated")
    jobs = [d for d in synth.config4() if d["fname"] == "log"]
    assert sorted(got) == [d["job_id"] for d in jobs]
    total = expect = 0
    for d in jobs:
        cases = got[d["job_id"]]
        assert len(cases) == len(set(cases)) and all(0 <= m < d["count"] for m in cases)
        job = Job(d["fname"], d["X0"], d["count"], d["s"], d["mode"], 1 << 16, 1 << 12, 3, 128)
        _check_cases(job, cases, sample=4)
        total += len(cases)
        expect += 2 * 2.0 ** -d["s"] * d["count"]
    assert expect / 4 < total < 4 * expect
