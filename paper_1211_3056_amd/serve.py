"""Serving loop: HR search jobs arriving over time, continuous batching.

Jobs (function, argument range, threshold) arrive at given times.  Each job
goes through
  queued   -> preparing (host tables in a worker process)
           -> ready     (waiting for device memory and a slot)
           -> admitted  (tables and items resident in HBM)
           -> done      (results read back, undecided values decided)
or failed (its preparation or launch raised; other jobs are unaffected).

Admission is by HBM footprint (tables + work items + a result reserve)
against a budget (default: the device's free memory) and by a cap on jobs
resident at once.  Every device step launches the fused persistent kernel
over the work items of all admitted jobs that have not run yet, so jobs that
arrived while others were on the GPU join the next launch (iteration-level
continuous batching); host preparation of arriving jobs overlaps device
work.  A job's results do not depend on which other jobs share its launch.

Preparation workers are processes started from a forkserver created before
the GPU is touched, so no process that has initialised the GPU forks or
execs.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import time
from dataclasses import dataclass, field

import numpy as np

from . import autotune
from .plan import ITEM_DTYPE, RESULT_DTYPE, BatchJob, plan_job, split_by_job
from .prep import JobSpec, SubPreparer, is_hr

RESULT_RESERVE = 64 * 32          # bytes reserved per job for its result records


@dataclass
class Prepared:
    """Host-side output of preparing one job (picklable)."""
    job: BatchJob
    delta: int
    W: int
    uf: str
    subs: list                    # (start, length, N)
    tables: np.ndarray            # uint64, concatenated sub-interval tables
    items: np.ndarray             # ITEM_DTYPE, table offsets relative to `tables`
    prep_s: float

    @property
    def footprint(self) -> int:
        return int(self.tables.nbytes + self.items.nbytes + RESULT_RESERVE)


def prepare_job(job: BatchJob, target_item_ns: float = 2000.0, part=None) -> Prepared:
    """Plan and prepare one job (runs in a worker process); part = (lo, hi)
    restricts it to sub-intervals lo..hi-1 (see merge_parts)."""
    t0 = time.time()
    pj = plan_job(job)
    sp = SubPreparer(job.fname, job.X0, job.s, job.mode, pj.delta, pj.W, pj.uf)
    tables, rows = [], []
    off = 0
    lo, hi = part if part is not None else (0, len(pj.subs))
    for t in range(lo, hi):
        s = pj.subs[t]
        table, win, thr = sp.prepare(s.start, s.length, s.N)
        cand = s.length * float(win[1]) / 2.0 ** 64
        last_piece = s.pieces - 1 if s.length % s.N else 0xFFFFFFFF
        last_N = s.length - (s.pieces - 1) * s.N
        for piece0, npieces, nu in autotune.split_sub(s.pieces, s.N, cand, target_item_ns):
            rows.append((off, int(win[0]), int(win[1]), tuple(int(x) for x in thr), job.job_id,
                         t, piece0, npieces, nu, s.N, last_piece, last_N))
        tables.append(table.reshape(-1))
        off += table.size
    return Prepared(job, pj.delta, pj.W, str(pj.uf),
                    [(s.start, s.length, s.N) for s in pj.subs[lo:hi]],
                    np.concatenate(tables), np.array(rows, dtype=ITEM_DTYPE), time.time() - t0)


def merge_parts(parts) -> Prepared:
    """One Prepared from the parts of a job prepared over consecutive
    sub-interval ranges, in order: tables concatenated, item table offsets
    moved accordingly (item sub indices are already global)."""
    if len(parts) == 1:
        return parts[0]
    items, base = [], 0
    for p in parts:
        it = p.items.copy()
        it["table"] += base
        base += p.tables.size
        items.append(it)
    p0 = parts[0]
    return Prepared(p0.job, p0.delta, p0.W, p0.uf, [s for p in parts for s in p.subs],
                    np.concatenate([p.tables for p in parts]), np.concatenate(items),
                    max(p.prep_s for p in parts))


def job_parts(job: BatchJob, subs_per_part: int):
    """Sub-interval ranges (lo, hi) of a job, for preparation by several
    workers; one range for jobs of at most subs_per_part sub-intervals."""
    n = -(-job.count // job.sub_len)
    if n <= subs_per_part:
        return [None]
    return [(lo, min(lo + subs_per_part, n)) for lo in range(0, n, subs_per_part)]


def decide_results(prep: Prepared, res: np.ndarray) -> np.ndarray:
    """Sorted HR offsets (int64 array) of one job from its result records."""
    from mpmath import mpf
    if len(res) == 0:
        return np.zeros(0, np.int64)
    starts = np.array([s[0] for s in prep.subs], dtype=np.int64)
    Ns = np.array([s[2] for s in prep.subs], dtype=np.int64)
    sub = res["sub"].astype(np.int64)
    m = starts[sub] + res["piece"].astype(np.int64) * Ns[sub] + res["k"].astype(np.int64)
    sure = m[res["cls"] == 1]
    und = m[res["cls"] == 2].tolist()
    if und:
        spec = JobSpec(prep.job.fname, prep.job.X0, prep.job.count, prep.job.s, prep.job.mode)
        uf = mpf(prep.uf)
        sure = np.concatenate([sure, np.array([x for x in und if is_hr(spec, x, uf)], np.int64)])
    return np.sort(sure)


@dataclass
class JobState:
    job: BatchJob
    arrival: float
    status: str = "queued"
    prep: Prepared | None = None
    t_ready: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    hr: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))   # sorted offsets
    records: np.ndarray | None = None   # result records, device order (plan.canonical sorts)
    error: str = ""
    dev: object = None            # device handle of the admitted job (backend-specific)
    parts: list = field(default_factory=list)   # prepared parts while preparing
    left: int = 0                 # parts still being prepared

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class GpuBackend:
    """Device side: uploads admitted jobs, launches the persistent kernel over
    their items, returns result records per job."""

    def __init__(self, cap: int = 1 << 20, waves: int | None = None):
        import torch

        from . import _lib, api
        from .batch import device_waves
        self.torch, self._lib, self.api = torch, _lib, api
        self.ctx = api.context()
        self.cap = cap
        self.waves = waves or device_waves()
        self.out = torch.empty(cap * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        self.count = torch.zeros(1, dtype=torch.uint64, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.uint64, device="cuda")
        self.steps = 0

    def free_memory(self) -> int:
        return int(self.torch.cuda.mem_get_info()[0])

    def admit(self, st: JobState):
        st.dev = self.api.to_dev(st.prep.tables, self.torch.uint64)

    def release(self, st: JobState):
        st.dev = None

    def step(self, states):
        """One launch over every item of the given admitted jobs; returns the
        result records of each job (list aligned with states)."""
        torch, _lib, api = self.torch, self._lib, self.api
        pool = torch.cat([s.dev for s in states])
        items, base = [], 0
        groups = {}
        for s in states:
            it = s.prep.items.copy()
            it["table"] += base
            base += s.prep.tables.size
            groups.setdefault((s.prep.W, s.prep.delta), []).append(it)
        launches = []
        for (W, d), parts in sorted(groups.items()):
            arr = np.concatenate(parts)
            launches.append((W, d, len(arr), api.to_dev(arr.view(np.uint8).reshape(-1), torch.uint8)))
        while True:
            self.count.zero_()
            for W, d, n_items, dev_items in launches:
                _lib.hr_batch_run(self.ctx, pool, dev_items, n_items, W, d, self.waves, self.out,
                                  self.cap, self.count, self.stats)
            torch.cuda.synchronize()
            n = api._u64_scalar(self.count)
            if n <= self.cap:
                break
            # more results than the buffer holds: grow it and run the step again
            self.cap = 1 << (n - 1).bit_length()
            self.out = torch.empty(self.cap * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        res = self.out[: n * _lib.RESULT_BYTES].cpu().numpy().view(RESULT_DTYPE)
        self.steps += 1
        return split_by_job(res, [s.job.job_id for s in states])


def make_pool(workers: int):
    """Process pool for host preparation; create it before the GPU is used."""
    ctx = mp.get_context("forkserver")
    pool = cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx)
    list(pool.map(_warm, range(workers)))
    return pool


def _warm(_):
    import mpmath  # noqa: F401
    return 0


class Server:
    """Continuous-batching server over a device backend."""

    def __init__(self, backend, pool, hbm_budget: int | None = None, max_resident: int = 4096,
                 clock=time.perf_counter, subs_per_part: int = 16):
        self.backend = backend
        self.pool = pool
        self.subs_per_part = subs_per_part   # large jobs are prepared by several workers
        self.budget = hbm_budget if hbm_budget is not None else int(0.9 * backend.free_memory())
        self.max_resident = max_resident
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.blocked_admissions = 0

    def serve(self, jobs, arrivals, realtime: bool = True, prepared=None):
        """Run every job; arrivals[i] is job i's arrival time in seconds from
        the start.  `prepared` (optional) maps job_id to a Prepared made
        ahead of time (cached tables): such jobs skip the worker pool.
        Returns the list of JobState in job order."""
        states = [JobState(j, float(a)) for j, a in zip(jobs, arrivals)]
        prepared = prepared or {}
        order = sorted(range(len(states)), key=lambda i: states[i].arrival)
        t0 = self.clock()
        now = lambda: self.clock() - t0
        nxt = 0
        futures = {}
        ready = []            # FIFO of prepared jobs waiting for admission
        resident = []         # admitted, not yet run
        done = 0
        while done < len(states):
            t = now()
            # arrivals -> preparation
            while nxt < len(order) and (not realtime or states[order[nxt]].arrival <= t):
                st = states[order[nxt]]
                nxt += 1
                if st.job.job_id in prepared:
                    st.prep = prepared[st.job.job_id]
                    st.status, st.t_ready = "ready", now()
                    ready.append(st)
                    continue
                st.status = "preparing"
                # split a large job over several workers only while workers
                # are idle: it cuts that job's latency, not the throughput
                idle = len(futures) < getattr(self.pool, "_max_workers", 1)
                parts = job_parts(st.job, self.subs_per_part) if idle else [None]
                st.parts, st.left = [None] * len(parts), len(parts)
                for i, part in enumerate(parts):
                    futures[self.pool.submit(prepare_job, st.job, 2000.0, part)] = (st, i)
            # finished preparations -> ready queue (arrival order kept by FIFO of completion)
            for fut in [f for f in futures if f.done()]:
                st, i = futures.pop(fut)
                if st.status == "failed":    # another part of it failed already
                    continue
                try:
                    st.parts[i] = fut.result()
                except Exception as e:       # a bad job fails alone
                    st.status, st.error, st.t_done = "failed", repr(e), now()
                    st.parts = []
                    done += 1
                    continue
                st.left -= 1
                if st.left == 0:
                    st.prep = merge_parts(st.parts)
                    st.parts = []
                    st.status = "ready"
                    st.t_ready = now()
                    ready.append(st)
            ready.sort(key=lambda s: s.arrival)
            # admission by footprint and resident slots
            while ready:
                st = ready[0]
                fp = st.prep.footprint
                if fp > self.budget:
                    ready.pop(0)
                    st.status, st.error, st.t_done = "failed", "job larger than the HBM budget", now()
                    done += 1
                    continue
                if self.used + fp > self.budget or len(resident) >= self.max_resident:
                    self.blocked_admissions += 1
                    break
                ready.pop(0)
                try:
                    self.backend.admit(st)
                except Exception as e:
                    st.status, st.error, st.t_done = "failed", repr(e), now()
                    done += 1
                    continue
                self.used += fp
                self.peak_used = max(self.peak_used, self.used)
                st.status, st.t_admit = "admitted", now()
                resident.append(st)
            # one device step over everything admitted
            if resident:
                batch, resident = resident, []
                try:
                    recs = self.backend.step(batch)
                except Exception as e:
                    recs = None
                    err = repr(e)
                for i, st in enumerate(batch):
                    if recs is None:
                        st.status, st.error = "failed", err
                    else:
                        st.records = recs[i]
                        st.hr = decide_results(st.prep, recs[i])
                        st.status = "done"
                    st.t_done = now()
                    self.used -= st.prep.footprint
                    self.backend.release(st)
                    done += 1
                continue
            if futures or nxt < len(order):
                # nothing to launch: wait for a preparation or the next arrival
                wait = 0.0005
                if not futures and nxt < len(order):
                    wait = max(0.0, states[order[nxt]].arrival - now())
                if futures:
                    cf.wait(list(futures), timeout=wait or 0.0005,
                            return_when=cf.FIRST_COMPLETED)
                else:
                    time.sleep(min(wait, 0.05))
        return states


def summarize(states, t_total: float | None = None):
    ok = [s for s in states if s.status == "done"]
    lat = np.array([s.latency for s in ok]) if ok else np.zeros(1)
    span = t_total if t_total is not None else (max(s.t_done for s in states) - min(s.arrival for s in states))
    n_args = sum(s.job.count for s in ok)
    return {"jobs": len(states), "done": len(ok), "failed": len(states) - len(ok),
            "makespan_s": span, "jobs_per_s": len(ok) / span, "args_per_s": n_args / span,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1000),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1000),
            "hr_cases": sum(len(s.hr) for s in ok)}
