"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

Shared by the tests, the bench and the oracle's callers.  Workloads are
shaped like the paper's (exp over binary64 sub-ranges of [1, 2), directed or
round-to-nearest HR thresholds), with random instances where the paper's
inputs are themselves arbitrary fractions.
"""
from __future__ import annotations

import numpy as np

# Plain degree-1 search: 4096 random (a, b), N = 2^16, threshold 2^-20.
CONFIG1 = dict(n=4096, N=1 << 16, D=1 << 44, seed=1)

# Plain pipeline, small: exp on [1, 1 + 2^-20) = 2^32 arguments, 256
# sub-intervals of 2^24, degree 3 at 192 bits, pieces of N = 2^16 (tau = 256),
# round-to-nearest, eps = 2^-24 ulp.
CONFIG2 = dict(fname="exp", X0=1.0, count=1 << 32, s=24, mode="rn",
               N=1 << 16, tau=1 << 8, delta=3, W=192)

# Plain pipeline, large: exp on [1, 1 + 2^-12) = 2^40 arguments, 4096
# sub-intervals of 2^28, degree 4 at 256 bits, N = 2^18 (tau = 1024),
# round-to-nearest, eps = 2^-32 ulp.
CONFIG3 = dict(fname="exp", X0=1.0, count=1 << 40, s=32, mode="rn",
               N=1 << 18, tau=1 << 10, delta=4, W=256)


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """numpy PCG64 generator for (seed, stream)."""
    return np.random.Generator(np.random.PCG64([seed, stream]) if stream else np.random.PCG64(seed))


def config1(seed: int = CONFIG1["seed"], n: int = CONFIG1["n"], N: int = CONFIG1["N"],
            D: int = CONFIG1["D"]):
    """(A, B, N[], D): A then B drawn uniformly from [0, 2^64)."""
    g = rng(seed)
    A = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    return A, B, np.full(n, N, np.uint32), D


def adversarial_instances(seed: int, n: int, max_N: int = 5000):
    """Instances hitting the degenerate corners: a = 0, powers of two, long
    runs of trailing zeros (short periods), a near 0 or 1, tiny and empty N,
    windows from empty to full."""
    g = rng(seed)
    A = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    kind = g.integers(0, 8, n)
    sh = g.integers(0, 64, n).astype(np.uint64)
    small = g.integers(0, 1000, n).astype(np.uint64)
    with np.errstate(over="ignore"):
        A = np.where(kind == 1, A >> sh, A)
        A = np.where(kind == 2, ~(A >> sh), A)
        A = np.where(kind == 3, small << sh, A)
        A = np.where(kind == 4, np.uint64(0), A)
        A = np.where(kind == 5, np.uint64(1) << sh, A)
    Nk = g.integers(0, 4, n)
    N = np.where(Nk == 0, g.integers(0, 4, n),
                 np.where(Nk == 1, g.integers(0, 300, n), g.integers(0, max_N, n))).astype(np.uint32)
    Dk = g.integers(0, 5, n)
    Dr = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    D = np.where(Dk == 0, Dr, np.where(Dk == 1, Dr >> sh, np.where(Dk == 2, np.uint64(2 ** 64 - 1),
                 np.where(Dk == 3, g.integers(0, 3, n).astype(np.uint64), np.uint64(1) << (sh | np.uint64(32))))))
    lo = np.where(g.integers(0, 2, n) == 0, np.uint64(0), g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False))
    return A, B, N, lo, D.astype(np.uint64)


def wave_slopes(seed: int, n_waves: int, N: int = 1 << 16, spread_log2: int = 34):
    """Instances in groups of 64 (one wave each) whose slopes are a base
    slope plus lane times 2^spread_log2 (as for adjacent pieces of one
    sub-interval), so that their leading partial quotients coincide; in
    every other group one lane gets an unrelated slope.  Base slopes are
    drawn in [1/3, 1), in (0, 1/3) and just above 1/2, b uniformly, N
    fixed, the threshold 2^-14.  Returns (A, B, N[], D)."""
    g = rng(seed)
    n = 64 * n_waves
    base = g.integers(0, 2 ** 64, n_waves, dtype=np.uint64, endpoint=False)
    kind = g.integers(0, 3, n_waves)
    third = np.uint64(0x5555555555555556)
    with np.errstate(over="ignore"):
        base = np.where(kind == 0, third + base % np.uint64(2 ** 64 - 0x5555555555555556 - 2 ** 41),
                        np.where(kind == 1, np.uint64(1) + base % (third - np.uint64(2 ** 41)),
                                 np.uint64(2 ** 63) + (base >> np.uint64(20))))
        A = np.repeat(base, 64) + (np.tile(np.arange(64, dtype=np.uint64), n_waves)
                                   << np.uint64(spread_log2))
    odd = np.arange(n_waves) % 2 == 1
    lane = g.integers(0, 64, n_waves)
    rand = g.integers(1, 2 ** 64, n_waves, dtype=np.uint64, endpoint=False)
    idx = (np.arange(n_waves) * 64 + lane)[odd]
    A[idx] = rand[odd]
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    return A, B, np.full(n, N, np.uint32), 1 << 50


def random_tables(seed: int, n_sub: int, delta: int, W: int):
    """Uniformly random initial tables: uint64 (n_sub, E, W/64)."""
    g = rng(seed)
    E = (delta + 1) * (delta + 2) // 2
    return g.integers(0, 2 ** 64, (n_sub, E, W // 64), dtype=np.uint64, endpoint=False)


# Batched form: 16 jobs, 4 per function, slices of 2^30 .. 2^38 arguments
# placed one after the other from each function's start, sub-intervals of
# 2^28 arguments with piece lengths N uniform in [2^12, 2^20], eps = 2^-28 RN.
CONFIG4 = dict(n_jobs=16, funcs=("exp", "log", "exp2", "sin"),
               starts={"exp": 1.0, "exp2": 1.0, "sin": 1.0, "log": 3.0},
               size_log2=(30, 38), N_range=(1 << 12, 1 << 20), s=28, sub_len=1 << 28, seed=4)


def _ulp(x: float) -> float:
    import math
    return math.ldexp(1.0, math.frexp(x)[1] - 53)


def config4(scale_log2: int = 0, N_scale_log2: int = 0, s: int | None = None, seed: int | None = None):
    """Job descriptions (dicts) of the batched workload.

    scale_log2 shrinks every slice and the sub-interval length by 2^scale_log2
    and N_scale_log2 the piece lengths (smaller copies of the same mix, for
    tests).  Job j is function funcs[j % 4]; its slice follows the previous
    slices of the same function.
    """
    c = CONFIG4
    g = rng(c["seed"] if seed is None else seed)
    gN = rng(c["seed"] if seed is None else seed, 2)
    lo, hi = c["size_log2"]
    sizes = g.integers(lo, hi + 1, c["n_jobs"])
    sub_len = c["sub_len"] >> scale_log2
    Nlo, Nhi = c["N_range"][0] >> N_scale_log2, c["N_range"][1] >> N_scale_log2
    used = {f: 0 for f in c["funcs"]}
    jobs = []
    for j in range(c["n_jobs"]):
        f = c["funcs"][j % len(c["funcs"])]
        count = 1 << (int(sizes[j]) - scale_log2)
        X0 = c["starts"][f] + used[f] * _ulp(c["starts"][f])
        used[f] += count
        n_sub = -(-count // sub_len)
        Ns = gN.integers(Nlo, Nhi, n_sub, endpoint=True).astype(int).tolist()
        jobs.append(dict(fname=f, X0=X0, count=count, s=c["s"] if s is None else s, mode="rn",
                         sub_len=sub_len, N=Ns, job_id=j))
    return jobs


# Serving: 2000 jobs, Poisson arrivals; f uniform over five functions, sizes
# round(2^U) with U ~ U(24, 36), eps 2^-20 or 2^-28, starts seeded and aligned
# to 2^24 arguments inside each function's one-binade region.
CONFIG5 = dict(n_jobs=2000, funcs=("exp", "log", "exp2", "sin", "cos"),
               starts={"exp": 1.0, "log": 3.0, "exp2": 1.0, "sin": 1.0, "cos": 1.0},
               # arguments available from the start with f in one output binade:
               # exp < ln 4, log < 4, 2^x < 2, sin < pi/2, cos > 1/2 (x < pi/3)
               room={"exp": 0.3862943611198906, "log": 1.0, "exp2": 1.0,
                     "sin": 0.5707963267948966, "cos": 0.0471975511965976},
               size_log2=(24.0, 36.0), s_choices=(20, 28), align=1 << 24, seed=5)


def config5(n_jobs: int | None = None, size_log2=None, seed: int | None = None):
    """Job descriptions (dicts) of the serving workload, in arrival order."""
    import math
    c = CONFIG5
    n = c["n_jobs"] if n_jobs is None else n_jobs
    lo, hi = c["size_log2"] if size_log2 is None else size_log2
    g = rng(c["seed"] if seed is None else seed)
    jobs = []
    for j in range(n):
        f = c["funcs"][int(g.integers(0, len(c["funcs"])))]
        size = int(round(2.0 ** g.uniform(lo, hi)))
        s = int(c["s_choices"][int(g.integers(0, len(c["s_choices"])))])
        h = _ulp(c["starts"][f])
        room_args = int(c["room"][f] / h) - size - 1
        slots = max(1, room_args // c["align"])
        off = int(g.integers(0, slots)) * c["align"]
        X0 = c["starts"][f] + off * h
        jobs.append(dict(fname=f, X0=X0, count=size, s=s, mode="rn", job_id=j))
    return jobs


def poisson_arrivals(n: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate (jobs/s)."""
    g = rng(seed, 2)
    return np.cumsum(g.exponential(1.0 / rate, n))
