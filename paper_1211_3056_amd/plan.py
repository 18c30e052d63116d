"""Torch-free planning of HR search jobs: sub-intervals, piece lengths,
degree and word width (autotuned when not given), and the device record
layouts shared by the batch runtime and the serving loop."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import autotune
from .prep import output_ulp_range

# hr_item and hr_result of include/hrsearch.h
ITEM_DTYPE = np.dtype([("table", np.uint64), ("win_lo", np.uint64), ("win_d", np.uint64),
                       ("thr", np.uint64, (4,)), ("job", np.uint32), ("sub", np.uint32),
                       ("piece0", np.uint32), ("npieces", np.uint32), ("nu", np.uint32),
                       ("N", np.uint32), ("last_piece", np.uint32), ("last_N", np.uint32)])
RESULT_DTYPE = np.dtype([("job", np.uint32), ("sub", np.uint32), ("piece", np.uint32),
                         ("k", np.uint32), ("cls", np.uint32), ("reserved", np.uint32),
                         ("value", np.uint64)])


@dataclass
class BatchJob:
    fname: str
    X0: float
    count: int
    s: int
    mode: str = "rn"
    sub_len: int = 1 << 28
    N: object = None          # int, list of ints (one per sub-interval), or None
    delta: int | None = None
    W: int | None = None
    job_id: int = 0


@dataclass
class PlannedSub:
    start: int
    length: int
    N: int

    @property
    def pieces(self) -> int:
        return -(-self.length // self.N)


@dataclass
class PlannedJob:
    job: BatchJob
    delta: int
    W: int
    uf: object
    subs: list = field(default_factory=list)


def plan_job(job: BatchJob) -> PlannedJob:
    uf = output_ulp_range(job.fname, job.X0, job.count)
    n_sub = -(-job.count // job.sub_len)
    if isinstance(job.N, (list, tuple, np.ndarray)):
        Ns = [int(x) for x in job.N]
        if len(Ns) != n_sub:
            raise ValueError("one N per sub-interval expected")
    else:
        N = int(job.N) if job.N else autotune.choose_N(job.fname, job.X0, job.count, job.s, uf)
        Ns = [N] * n_sub
    subs = []
    for t in range(n_sub):
        start = t * job.sub_len
        length = min(job.sub_len, job.count - start)
        subs.append(PlannedSub(start, length, min(Ns[t], length)))
    delta = job.delta or autotune.choose_degree(job.fname, job.X0, job.sub_len, job.s, uf)
    W = job.W or autotune.choose_width([(s.N, s.pieces) for s in subs], delta, job.s)
    for s in subs:
        if s.pieces ** delta >= 1 << 128 or s.N ** delta >= 1 << 128:
            raise ValueError("piece count or length too large for the degree")
    return PlannedJob(job, delta, W, uf, subs)
