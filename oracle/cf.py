"""Continued fractions and two-length configurations (oracle).

Follows Sec. 3.2 of the paper ("Properties of the set {a x mod 1 | x < n}"):
the Euclidean remainders theta_i, the convergent denominators q_i, the partial
quotients k_{i+1} = floor(theta_{i-1} / theta_i), the intermediate lengths
theta_{i-1,t} = theta_{i-1} - t theta_i and counts q_{i-1,t} = q_{i-1} + t q_i
(t in [0, k_{i+1})), Eq. 2 (q_i theta_{i-1,t} + q_{i-1,t} theta_i = 1), and the
two-length configuration labels (i, t) of Table 2 / Fig. 3.

Everything is exact integer arithmetic over a generic modulus M: a real a in
[0, 1) is the rational A / M, lengths are scaled by M (as Table 2 scales by 45),
so Eq. 2 reads q_i theta_{i-1,t} + q_{i-1,t} theta_i = M.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass
class Expansion:
    """Euclid sequences of A/M, indexed from -1 (the paper's initial values).

    theta[i+1], q[i+1], p[i+1] hold theta_i, q_i, p_i for i >= -1, and
    k[i+1] holds k_{i+1} (k[0] is unused).
    """

    theta: list
    q: list
    p: list
    k: list

    def th(self, i):
        return self.theta[i + 1]

    def qq(self, i):
        return self.q[i + 1]

    def kk(self, i):
        """k_i (the i-th partial quotient, i >= 1)."""
        return self.k[i]


def expansion(A: int, M: int) -> Expansion:
    """Remainders, convergents and quotients of A/M (Sec. 3.2 recurrences).

    p_{-1}=1, p_0=0, q_{-1}=0, q_0=1, theta_{-1}=1 (scaled: M), theta_0=a (A);
    k_{i+1} = floor(theta_{i-1}/theta_i), theta_{i+1} = theta_{i-1} - k_{i+1}
    theta_i, and the same recurrence for p and q.  Stops after the remainder
    reaches 0 (A/M is rational, Sec. 3.2 last paragraph).
    """
    if not (0 <= A < M):
        raise ValueError("need 0 <= A < M")
    theta = [M, A]
    q = [0, 1]
    p = [1, 0]
    k = [None]
    while theta[-1] != 0:
        kk = theta[-2] // theta[-1]
        k.append(kk)
        theta.append(theta[-2] - kk * theta[-1])
        q.append(q[-2] + kk * q[-1])
        p.append(p[-2] + kk * p[-1])
    return Expansion(theta, q, p, k)


def two_length_configs(A: int, M: int):
    """Rows (i, t, q_{i-1,t}, q_i, theta_{i-1,t}, theta_i, k_{i+1}) of Table 2.

    One row per two-length configuration (i, t), t in [0, k_{i+1}), for every
    i with theta_i != 0, followed by the terminal row (i, 0) with theta_i = 0
    (Table 2's last row; its k column is a placeholder and is reported here as
    None).
    """
    e = expansion(A, M)
    rows = []
    i = 0
    while True:
        th_i = e.th(i)
        q_i = e.qq(i)
        if th_i == 0:
            rows.append((i, 0, e.qq(i - 1), q_i, e.th(i - 1), 0, None))
            break
        k_next = e.kk(i + 1)
        for t in range(k_next):
            rows.append((i, t, e.qq(i - 1) + t * q_i, q_i,
                         e.th(i - 1) - t * th_i, th_i, k_next))
        i += 1
    return rows


def points(A: int, M: int, n: int):
    """Sorted positions {x A mod M | 0 <= x < n} (scaled by M)."""
    return sorted((x * A) % M for x in range(n))


def gap_sequence(A: int, M: int, n: int):
    """Lengths of the n intervals cut by n points, left to right from 0.

    This is what Fig. 3 prints on each line (one line per n), the last gap
    running from the largest point to M (the unit segment's end).
    """
    pos = points(A, M, n)
    return [b - a for a, b in zip(pos, pos[1:] + [M])]


def config_points(A: int, M: int, i: int, t: int) -> int:
    """Number of points q_i + q_{i-1,t} of configuration (i, t) (Eq. 2)."""
    e = expansion(A, M)
    return e.qq(i) + e.qq(i - 1) + t * e.qq(i)
