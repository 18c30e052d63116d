"""The packet start used by the tabulation kernels, checked in exact integers.

A lane starting at piece x needs the differences of its row with step H
(H = 32 in hr_tabulate, 64 in the fused pass).  The kernels form them in
one pass from the sub-interval's step-1 differences at piece 0:

    Delta_H^m r(x) = sum_{n >= m} c[m][n] Delta^n r(0),
    c[m][n] = sum_{k=m..n} A[m][k] C(x, n - k),

with A the coefficients of (E^H - 1)^m in powers of Delta (the straightforward
shift of Sec. 5.2 composed with the change of step), and use 64-bit
multipliers when x + D H is below the 64-bit binomial limit of the degree D.
These tests check the identity against differences taken directly, the bound
c[m][n] <= C(x + m H, n) that the kernels rely on, and that the bound keeps
every multiplier and every term below 2^64 right up to the limit.
"""
from math import comb

import pytest

import synth

# largest x with x (x - 1) .. (x - D + 1) < 2^64 that the kernels accept, by
# degree (the limit is exclusive)
LIMIT64 = {1: 1 << 32, 2: 1 << 32, 3: 1 << 21, 4: 1 << 16, 5: 1 << 12, 6: 1 << 10}


def step_coefficients(H, D):
    """A[m][k]: (E^H - 1)^m = sum_k A[m][k] Delta^k, from E^H - 1 =
    sum_{i>=1} C(H, i) Delta^i."""
    A = [[0] * (D + 1) for _ in range(D + 1)]
    A[0][0] = 1
    for m in range(1, D + 1):
        for k in range(m, D + 1):
            A[m][k] = sum(A[m - 1][k - i] * comb(H, i) for i in range(1, k - m + 2))
    return A


def composed(H, D, x):
    A = step_coefficients(H, D)
    return [[sum(A[m][k] * comb(x, n - k) for k in range(m, n + 1)) if n >= m else 0
             for n in range(D + 1)] for m in range(D + 1)]


def differences(f, x, h, D):
    """Delta_h^m f(x), m = 0..D, from D + 1 values of f."""
    vals = [f(x + i * h) for i in range(D + 1)]
    out = []
    for _ in range(D + 1):
        out.append(vals[0])
        vals = [vals[i + 1] - vals[i] for i in range(len(vals) - 1)]
    return out


@pytest.mark.parametrize("H", [32, 64])
@pytest.mark.parametrize("D", [1, 2, 3, 4, 5, 6])
def test_composed_start_equals_direct_differences(H, D):
    g = synth.rng(1000 * H + D)
    for _ in range(12):
        co = [int(v) - (1 << 62) for v in g.integers(0, 1 << 63, D + 1, dtype="uint64")]
        f = lambda t: sum(c * t ** i for i, c in enumerate(co))   # noqa: E731
        T = differences(f, 0, 1, D)
        x = int(g.integers(0, 5000))
        c = composed(H, D, x)
        got = [sum(c[m][n] * T[n] for n in range(m, D + 1)) for m in range(D + 1)]
        assert got == differences(f, x, H, D)
        for m in range(D + 1):
            assert c[m][m] == H ** m          # the diagonal is a shift


@pytest.mark.parametrize("H", [32, 64])
@pytest.mark.parametrize("D", [1, 2, 3, 4, 5, 6])
def test_multiplier_bound_and_64_bit_range(H, D):
    A = step_coefficients(H, D)
    top = LIMIT64[D] - 1 - D * H          # largest first piece of the 64-bit path
    if top < 0:
        pytest.skip("no first piece fits below the limit at this degree and step")
    for x in sorted({0, 1, 2, H - 1, top // 2, top}):
        c = composed(H, D, x)
        for m in range(D + 1):
            for n in range(m, D + 1):
                assert 0 <= c[m][n] <= comb(x + m * H, n)
                assert c[m][n] < 1 << 64
                for k in range(m, n + 1):
                    assert A[m][k] * comb(x, n - k) < 1 << 64
