"""Torch-free planning of HR search jobs: sub-intervals, piece lengths,
degree and word width (autotuned when not given), the upper tables, windows
and work items the device needs, and the device record layouts shared by
the batch runtime and the serving loop."""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import math
import time

from . import autotune
from .prep import (MAX_UPPER_DEGREE, output_ulp_range, upper_error, upper_table,
                   upper_windows_many)

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


# ---------------------------------------------------------------- device-made tables

def upper_ranges(pj: PlannedJob, Wu: int | None = None):
    """Cut a planned job into ranges of whole sub-intervals, each covered by
    one upper polynomial (the smallest degree >= delta whose Lagrange
    remainder over the range is below eps 2^-12, at most MAX_UPPER_DEGREE;
    a range that needs more is halved), at the narrowest width that suits it
    (autotune.choose_upper_width) unless Wu is given.  Returns
    [(t_lo, t_hi, UpperTable)]."""
    job = pj.job
    lim = 2.0 ** (-job.s - autotune.MARGIN_BITS)
    h = math.ldexp(1.0, math.frexp(job.X0)[1] - 53)
    out = []
    todo = [(0, len(pj.subs))]
    while todo:
        lo, hi = todo.pop(0)
        start = pj.subs[lo].start
        count = pj.subs[hi - 1].start + pj.subs[hi - 1].length - start
        X0 = job.X0 + start * h
        Du = next((d for d in range(max(pj.delta, 1), MAX_UPPER_DEGREE + 1)
                   if float(upper_error(job.fname, X0, count, d, pj.uf)) <= lim), None)
        if Du is None:
            if hi - lo == 1:
                raise ValueError("sub-interval too long for an upper polynomial")
            mid = (lo + hi) // 2
            todo[:0] = [(lo, mid), (mid, hi)]
            continue
        width = Wu or autotune.choose_upper_width(
            Du, hi - lo, max(sp.N for sp in pj.subs[lo:hi]),
            max(sp.pieces for sp in pj.subs[lo:hi]), pj.delta, job.s)
        U = upper_table(job.fname, X0, count, job.s, job.mode, job.sub_len, Du, width, uf=pj.uf)
        out.append((lo, hi, U))
    return out


@dataclass
class TablePlan:
    """What the device needs to make and search one job's tables (picklable):
    the upper tables of its ranges, the piece length of every sub-interval,
    the shared windows and thresholds, and the work items.  Item table
    offsets are relative to the job's own table region (sub-interval t's
    table at t E W/64 words)."""
    job: BatchJob
    delta: int
    W: int
    uf: str
    subs: list                    # (start, length, N) per sub-interval
    ranges: list                  # (t_lo, t_hi, Du, Wu, words uint64 (E_u, Wu/64))
    Ns: np.ndarray                # uint32, piece length per sub-interval
    win: np.ndarray               # uint64 (n_sub, 2)
    thr: np.ndarray               # uint64 (n_sub, 4)
    items: np.ndarray             # ITEM_DTYPE
    prep_s: float = 0.0

    @property
    def entries(self) -> int:
        return (self.delta + 1) * (self.delta + 2) // 2

    @property
    def table_words(self) -> int:
        return len(self.subs) * self.entries * (self.W // 64)

    @property
    def footprint(self) -> int:
        """Device bytes while resident: the tables, the upper tables, the
        piece lengths and the work items."""
        return int(self.table_words * 8 + sum(r[4].nbytes for r in self.ranges)
                   + self.Ns.nbytes + self.items.nbytes)


def job_windows(pj: PlannedJob, ranges):
    """Windows and thresholds of every sub-interval (one vectorised bound
    per range over its sub-intervals' (N, pieces))."""
    n = len(pj.subs)
    win = np.zeros((n, 2), np.uint64)
    thr = np.zeros((n, 4), np.uint64)
    for lo, hi, U in ranges:
        Ns = [pj.subs[t].N for t in range(lo, hi)]
        taus = [pj.subs[t].pieces for t in range(lo, hi)]
        win[lo:hi], thr[lo:hi] = upper_windows_many(U, Ns, taus, pj.delta, pj.W)
    return win, thr


def job_items(pj: PlannedJob, win, thr, target_ns: float, model=autotune.MODEL):
    """Work items of one job (table offsets relative to its table region)."""
    E = (pj.delta + 1) * (pj.delta + 2) // 2
    L = pj.W // 64
    rows = []
    for t, sp in enumerate(pj.subs):
        cand = sp.length * float(win[t, 1]) / 2.0 ** 64
        last_piece = sp.pieces - 1 if sp.length % sp.N else 0xFFFFFFFF
        last_N = sp.length - (sp.pieces - 1) * sp.N
        th = tuple(int(x) for x in thr[t])
        for piece0, npieces, nu in autotune.split_sub(sp.pieces, sp.N, cand, target_ns, model):
            rows.append((t * E * L, int(win[t, 0]), int(win[t, 1]), th, pj.job.job_id, t,
                         piece0, npieces, nu, sp.N, last_piece, last_N))
    return np.array(rows, dtype=ITEM_DTYPE)


def sub_costs(pj: PlannedJob, win, model=autotune.MODEL) -> float:
    """Modelled device time of a job (ns), from its windows."""
    return sum(model.cost(sp.pieces, sp.N, sp.length * float(win[t, 1]) / 2.0 ** 64)
               for t, sp in enumerate(pj.subs))


def plan_tables(job: BatchJob, target_ns: float | None = None, model=autotune.MODEL,
                target_items: int = 16) -> TablePlan:
    """Plan one job for device-made tables.  Items are split to about
    target_ns of modelled work each (default: the job's cost over
    target_items)."""
    t0 = time.time()
    pj = plan_job(job)
    ranges = upper_ranges(pj)
    win, thr = job_windows(pj, ranges)
    if target_ns is None:
        target_ns = max(sub_costs(pj, win, model) / target_items, 1e-9)
    items = job_items(pj, win, thr, target_ns, model)
    return TablePlan(job, pj.delta, pj.W, str(pj.uf),
                     [(sp.start, sp.length, sp.N) for sp in pj.subs],
                     [(lo, hi, U.Du, U.Wu, U.words) for lo, hi, U in ranges],
                     np.array([sp.N for sp in pj.subs], np.uint32), win, thr, items,
                     time.time() - t0)
