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


def split_by_job(res: np.ndarray, job_ids):
    """Result records of each job, in job_ids order; within a job the records
    keep their device order (see canonical()).  One stable 16-bit radix sort
    of the step's records by local job index, then contiguous slices."""
    ids = np.asarray(job_ids, dtype=np.int64)
    if ids.size == 0:
        return []
    if ids.size >= 1 << 16:
        raise ValueError("too many jobs in one step")
    job = res["job"].astype(np.int64)
    other = ids.size                                   # bucket of unknown job ids
    if ids.max() < 1 << 24:
        lut = np.full(int(ids.max()) + 2, other, dtype=np.int64)
        lut[ids] = np.arange(ids.size)
        local = lut[np.minimum(job, ids.max() + 1)]
    else:
        srt = np.argsort(ids)
        pos = np.minimum(np.searchsorted(ids[srt], job), ids.size - 1)
        local = np.where(ids[srt][pos] == job, srt[pos], other)
    local = local.astype(np.uint16)
    order = np.argsort(local, kind="stable")
    bounds = np.concatenate([[0], np.cumsum(np.bincount(local, minlength=other + 1))])
    # gather whole 32-byte records as rows of 4 uint64 (a structured gather is
    # several times slower)
    rows = np.take(np.ascontiguousarray(res).view(np.uint64).reshape(-1, 4), order, axis=0)
    res = rows.reshape(-1).view(RESULT_DTYPE)
    return [res[bounds[i]:bounds[i + 1]] for i in range(ids.size)]


def canonical(records: np.ndarray) -> np.ndarray:
    """Records sorted by (job, sub, piece, k): a device-order-free form."""
    return records[np.lexsort((records["k"], records["piece"], records["sub"], records["job"]))]
