"""Pins for oracle/cf.py: Table 2, Fig. 3, Eq. 2, Props. 1-2 (Sec. 3.2)."""
import random

import pytest

from oracle import cf
from tests.conftest import read_golden


def _table2():
    rows = []
    for line in read_golden("table2_a14_m45.txt"):
        f = line.split()
        rows.append(tuple(int(x) for x in f[:6]) + (None if f[6] == "-" else int(f[6]),))
    return rows


def test_table2_exact():
    assert cf.two_length_configs(14, 45) == _table2()


def test_cf_of_14_45():
    e = cf.expansion(14, 45)
    assert e.k[1:] == [3, 4, 1, 2]                      # 14/45 = [0; 3, 4, 1, 2]
    assert e.theta == [45, 14, 3, 2, 1, 0]
    assert e.q == [0, 1, 3, 13, 16, 45]


def _fig3():
    out = {}
    for line in read_golden("fig3_gaps_a14_m45.txt"):
        head, gaps = line.split("|")
        n, label = head.split()
        out[int(n)] = (label, [int(g) for g in gaps.split()])
    return out


def test_fig3_gap_sequences():
    for n, (_, gaps) in _fig3().items():
        assert cf.gap_sequence(14, 45, n) == gaps, n


def test_fig3_labels_are_two_length_configs():
    """Lines labelled (i, t) hold q_i + q_{i-1,t} points, and only there does
    the configuration have exactly two lengths in the proportions of Eq. 2."""
    fig = _fig3()
    rows = cf.two_length_configs(14, 45)
    labelled = {(r[0], r[1]): r[2] + r[3] for r in rows}
    for n, (label, gaps) in fig.items():
        if label == "-":
            continue
        i, t = (int(x) for x in label.strip("()").split(","))
        assert labelled[(i, t)] == n
        row = [r for r in rows if (r[0], r[1]) == (i, t)][0]
        _, _, q_it, q_i, th_it, th_i, _ = row
        # q_i intervals of length theta_{i-1,t} and q_{i-1,t} of length theta_i
        if th_i == th_it:
            assert gaps.count(th_i) == q_i + q_it
        else:
            assert gaps.count(th_it) == q_i
            assert gaps.count(th_i) == q_it
            assert len(set(gaps)) <= 2


def test_eq2_identity_random_64bit():
    """q_i theta_{i-1,t} + q_{i-1,t} theta_i = 1 (scaled: 2^64), every (i, t)."""
    rng = random.Random(7)
    M = 1 << 64
    for _ in range(200):
        A = rng.randrange(1, M)
        for (i, t, q_it, q_i, th_it, th_i, _) in cf.two_length_configs(A, M)[:60]:
            assert q_i * th_it + q_it * th_i == M


@pytest.mark.parametrize("M", [45, 97, 1 << 10, 3 ** 7])
def test_two_length_property_bruteforce(M):
    """At every (i, t) the n = q_i + q_{i-1,t} points cut exactly q_i
    intervals of length theta_{i-1,t} and q_{i-1,t} of length theta_i."""
    rng = random.Random(M)
    for _ in range(25):
        A = rng.randrange(1, M)
        for (i, t, q_it, q_i, th_it, th_i, _) in cf.two_length_configs(A, M):
            if th_i == 0:
                continue
            gaps = cf.gap_sequence(A, M, q_i + q_it)
            expect = {}
            for length, cnt in ((th_it, q_i), (th_i, q_it)):
                if cnt:
                    expect[length] = expect.get(length, 0) + cnt
            assert {g: gaps.count(g) for g in set(gaps)} == expect


def test_prop2_directed_reduction():
    """Going from (i, t) to (i, t+1), each theta_{i-1,t} interval is split into
    (theta_i, theta_{i-1,t+1}) left to right for even i, reversed for odd i."""
    rng = random.Random(3)
    M = 1 << 12
    checked = 0
    for _ in range(40):
        A = rng.randrange(1, M)
        rows = cf.two_length_configs(A, M)
        for r0, r1 in zip(rows, rows[1:]):
            i, t, q_it, q_i, th_it, th_i, _ = r0
            if th_i == 0 or r1[5] == 0 or th_it == th_i:
                continue
            before = cf.points(A, M, q_i + q_it)
            after = cf.points(A, M, r1[2] + r1[3])
            new_len = th_it - th_i          # theta_{i-1,t+1} (or theta_{i+1})
            for lo, hi in zip(before, before[1:] + [M]):
                if hi - lo != th_it:
                    continue
                inside = [p for p in after if lo < p < hi]
                assert len(inside) == 1
                left = inside[0] - lo
                if i % 2 == 0:
                    assert (left, hi - inside[0]) == (th_i, new_len)
                else:
                    assert (left, hi - inside[0]) == (new_len, th_i)
                checked += 1
    assert checked > 100


def test_prop1_next_configuration():
    """Consecutive labels follow (i, t) -> (i, t+1) or (i+1, 0)."""
    M = 1 << 16
    rng = random.Random(11)
    for _ in range(50):
        rows = cf.two_length_configs(rng.randrange(1, M), M)
        for r0, r1 in zip(rows, rows[1:]):
            i, t, *_, k = r0
            if t < k - 1:
                assert (r1[0], r1[1]) == (i, t + 1)
            else:
                assert (r1[0], r1[1]) == (i + 1, 0)


def test_config_points_gives_two_length_configurations():
    """config_points(i, t) = q_i + q_{i-1,t} (Eq. 2): the brute-force point
    set of that size has exactly the two lengths theta_i and theta_{i-1,t}
    (Sec. 3.2), for Table 2's a = 14/45 and random fractions.  A count off
    by one point, or without the t q_i term, yields three lengths."""
    rng = random.Random(31)
    cases = [(14, 45)] + [(rng.randrange(1, M), M) for M in (97, 1000, 4096, 65537)
                          for _ in range(12)]
    checked = 0
    for A, M in cases:
        e = cf.expansion(A, M)
        i = 0
        while e.th(i) != 0 and e.qq(i) + e.qq(i - 1) <= 3000:
            for t in range(min(e.kk(i + 1), 6)):
                n = cf.config_points(A, M, i, t)
                if n > 3000:
                    break
                lengths = set(cf.gap_sequence(A, M, n))
                assert lengths <= {e.th(i), e.th(i - 1) - t * e.th(i)}, (A, M, i, t)
                checked += 1
            i += 1
    assert checked > 200
