"""Serving loop: HR search jobs arriving over time, continuous batching.

Jobs (function, argument range, threshold) arrive at given times.  Each job
goes through
  queued   -> preparing (upper tables, windows and work items, in a worker
              process)
           -> ready     (waiting for device memory and a slot)
           -> admitted  (its sub-interval tables made on the device, from
                         its upper tables, in its region of the table arena)
           -> done      (results read back, undecided values decided)
or failed (its preparation or launch raised; other jobs are unaffected).

Admission is by HBM footprint (tables, upper tables and work items) against
a budget (default: the arena's size, at most 90% of the device's free
memory) and by a cap on jobs resident at once.  Admitted tables live in one
device arena at offsets from a free list, so a step needs no copy of them.
Every device step launches the fused persistent kernel over the work items
of all admitted jobs that have not run yet, so jobs that arrived while
others were on the GPU join the next launch (iteration-level continuous
batching); host preparation of arriving jobs overlaps device work.  A job's
results do not depend on which other jobs share its launch.

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

from .plan import ITEM_DTYPE, RESULT_DTYPE, BatchJob, TablePlan, plan_tables, split_by_job  # noqa: F401
from .prep import JobSpec, is_hr

Prepared = TablePlan


def prepare_job(job: BatchJob, target_item_ns: float = 2000.0) -> TablePlan:
    """Plan and prepare one job (runs in a worker process)."""
    return plan_tables(job, target_item_ns)


def decide_results(prep: TablePlan, res: np.ndarray) -> np.ndarray:
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


class Arena:
    """First-fit allocator of word ranges [offset, offset + n) in one device
    buffer of `words` words; freed ranges merge with free neighbours."""

    def __init__(self, words: int):
        self.words = words
        self.free = [(0, words)]          # sorted, disjoint (offset, length)

    def alloc(self, n: int):
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                return off
        return None

    def release(self, off: int, n: int):
        import bisect
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, n))
        if i + 1 < len(self.free) and off + n == self.free[i + 1][0]:
            self.free[i] = (off, n + self.free.pop(i + 1)[1])
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            po, pn = self.free.pop(i - 1)
            self.free[i - 1] = (po, pn + self.free[i - 1][1])

    @property
    def free_words(self) -> int:
        return sum(n for _, n in self.free)


@dataclass
class JobState:
    job: BatchJob
    arrival: float
    status: str = "queued"
    prep: TablePlan | None = None
    t_ready: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    hr: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))   # sorted offsets
    records: np.ndarray | None = None   # result records, device order (plan.canonical sorts)
    error: str = ""
    dev: object = None            # device handle of the admitted job (backend-specific)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class GpuBackend:
    """Device side: makes admitted jobs' tables in the arena, launches the
    persistent kernel over their items, returns result records per job."""

    def __init__(self, cap: int = 1 << 20, waves: int | None = None, arena_bytes: int = 1 << 30,
                 slots: int = 4):
        import torch

        from . import _lib, api
        from .batch import device_waves
        self.torch, self._lib, self.api = torch, _lib, api
        self.ctx = api.context()
        self.cap = cap
        self.waves = waves or device_waves()
        self.arena_t = torch.empty(arena_bytes // 8, dtype=torch.uint64, device="cuda")
        self.arena = Arena(arena_bytes // 8)
        self.capacity_bytes = arena_bytes
        self.out = torch.empty(cap * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        self.count = torch.zeros(1, dtype=torch.uint64, device="cuda")
        self.stats = torch.zeros(8, dtype=torch.uint64, device="cuda")
        self.steps = 0
        self.slots = slots
        self.stream_b = None             # the hr_batch stream, opened on first use
        self.inflight = {}               # ticket -> (states, item lists, result buffers)

    def free_memory(self) -> int:
        return int(self.torch.cuda.mem_get_info()[0])

    def admit(self, st: JobState) -> bool:
        """Make the job's tables in a region of the arena; False (nothing
        done) if no free range is long enough."""
        from .batch import make_tables
        off = self.arena.alloc(st.prep.table_words)
        if off is None:
            return False
        try:
            make_tables(self.ctx, self.arena_t, off, st.prep)
        except Exception:
            self.arena.release(off, st.prep.table_words)
            raise
        st.dev = off
        return True

    def release(self, st: JobState):
        if st.dev is not None:
            self.arena.release(st.dev, st.prep.table_words)
            st.dev = None

    def _items(self, states):
        """Device item lists of the given admitted jobs, one per (W, delta)."""
        torch, api = self.torch, self.api
        groups = {}
        for s in states:
            it = s.prep.items.copy()
            it["table"] += s.dev
            groups.setdefault((s.prep.W, s.prep.delta), []).append(it)
        out = []
        for (W, d), parts in sorted(groups.items()):
            arr = np.concatenate(parts)
            out.append((W, d, len(arr), api.to_dev(arr.view(np.uint8).reshape(-1), torch.uint8)))
        return out

    def _run_sync(self, launches):
        """Run item lists with hr_batch_run, growing the result buffer until
        every record fits; returns the records."""
        torch, _lib, api = self.torch, self._lib, self.api
        while True:
            self.count.zero_()
            for W, d, n_items, dev_items in launches:
                _lib.hr_batch_run(self.ctx, self.arena_t, dev_items, n_items, W, d, self.waves,
                                  self.out, self.cap, self.count, self.stats)
            torch.cuda.synchronize()
            n = api._u64_scalar(self.count)
            if n <= self.cap:
                break
            # more results than the buffer holds: grow it and run again
            self.cap = 1 << (n - 1).bit_length()
            self.out = torch.empty(self.cap * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        return self.out[: n * _lib.RESULT_BYTES].cpu().numpy().view(RESULT_DTYPE).copy()

    def step(self, states):
        """One launch over every item of the given admitted jobs, waited
        for; returns the result records of each job (aligned with states)."""
        res = self._run_sync(self._items(states))
        self.steps += 1
        return split_by_job(res, [s.job.job_id for s in states])

    # ---- streamed launches (hr_batch_*): submit returns at once, collect
    # hands back the launches that have completed

    def submit(self, states):
        """Queue one launch over the given admitted jobs on the batch stream
        (after the work queued so far on the current stream, which made their
        tables); returns a ticket, or None while no launch slot is free."""
        torch, _lib = self.torch, self._lib
        if self.stream_b is None:
            self.stream_b = _lib.BatchStream(self.ctx, slots=self.slots)
            self.free_bufs = [(torch.empty(self.cap * _lib.RESULT_BYTES, dtype=torch.uint8,
                                           device="cuda"),
                               torch.zeros(1, dtype=torch.uint64, device="cuda"), self.cap)
                              for _ in range(self.slots)]
        launches = self._items(states)
        if len(launches) != 1 or not self.free_bufs:
            return None                  # several (W, delta) groups: run them synchronously
        W, d, n_items, dev_items = launches[0]
        out, count, cap = self.free_bufs[-1]
        t = self.stream_b.submit(self.arena_t, dev_items, n_items, W, d, out, cap, count,
                                 after_stream=torch.cuda.current_stream())
        if t is None:
            return None
        self.free_bufs.pop()
        self.inflight[t] = (states, launches, (out, count, cap))
        self.steps += 1
        return t

    def wait_oldest(self):
        """Block until the oldest launch in flight is over."""
        if self.inflight:
            self.stream_b.wait(min(self.inflight))

    def collect(self):
        """[(states, records per job)] of every submitted launch that has
        completed, in ticket order."""
        api, _lib = self.api, self._lib
        if not self.inflight:
            return []
        done = self.stream_b.poll()
        out = []
        for t in sorted(k for k in self.inflight if k <= done):
            states, launches, (buf, count, cap) = self.inflight.pop(t)
            n = api._u64_scalar(count)
            if n <= cap:
                res = buf[: n * _lib.RESULT_BYTES].cpu().numpy().view(RESULT_DTYPE).copy()
            else:                        # the buffer was too small: run it again, waited for
                res = self._run_sync(launches)
            self.free_bufs.append((buf, count, cap))
            out.append((states, split_by_job(res, [s.job.job_id for s in states])))
        return out


def make_pool(workers: int):
    """Process pool for host preparation; create it before the GPU is used."""
    ctx = mp.get_context("forkserver")
    pool = cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx)
    list(pool.map(_warm, range(workers)))
    return pool


def _warm(_):
    import mpmath  # noqa: F401

    from . import plan  # noqa: F401
    return 0


class Server:
    """Continuous-batching server over a device backend."""

    def __init__(self, backend, pool, hbm_budget: int | None = None, max_resident: int = 4096,
                 clock=time.perf_counter):
        self.backend = backend
        self.pool = pool
        cap = getattr(backend, "capacity_bytes", None)
        budget = int(0.9 * backend.free_memory())
        if cap is not None:
            budget = min(budget, cap)
        self.budget = hbm_budget if hbm_budget is not None else budget
        self.max_resident = max_resident
        self.clock = clock
        self.used = 0
        self.peak_used = 0
        self.blocked_admissions = 0

    def _finish(self, batch, recs, err, now):
        """Mark a launched batch done (or failed), release its memory;
        returns the number of jobs."""
        return _finish_batch(self, batch, recs, err, now)

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
                futures[self.pool.submit(prepare_job, st.job, 2000.0)] = st
            # finished preparations -> ready queue
            for fut in [f for f in futures if f.done()]:
                st = futures.pop(fut)
                try:
                    st.prep = fut.result()
                except Exception as e:       # a bad job fails alone
                    st.status, st.error, st.t_done = "failed", repr(e), now()
                    done += 1
                    continue
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
                try:
                    placed = self.backend.admit(st)
                except Exception as e:
                    ready.pop(0)
                    st.status, st.error, st.t_done = "failed", repr(e), now()
                    done += 1
                    continue
                if placed is False:          # no free range long enough yet
                    if self.used == 0:           # and nothing will free one
                        ready.pop(0)
                        st.status, st.t_done = "failed", now()
                        st.error = "job larger than the table arena"
                        done += 1
                        continue
                    self.blocked_admissions += 1
                    break
                ready.pop(0)
                self.used += fp
                self.peak_used = max(self.peak_used, self.used)
                st.status, st.t_admit = "admitted", now()
                resident.append(st)
            streamed = hasattr(self.backend, "submit")
            progressed = False
            # launch everything admitted: queued at once on the batch stream
            # (streamed backends), else one waited-for step
            if resident:
                batch, recs, err = resident, None, ""
                if streamed:
                    try:
                        ticket = self.backend.submit(batch)
                    except Exception as e:
                        ticket, err = None, repr(e)
                    if ticket is not None:
                        resident = []
                        progressed = True
                        batch = None
                if batch is not None and (not streamed or err or not self.backend.inflight):
                    resident = []
                    if not err:
                        try:
                            recs = self.backend.step(batch)
                        except Exception as e:
                            err = repr(e)
                    done += self._finish(batch, recs, err, now)
                    progressed = True
            if streamed:
                for batch, recs in self.backend.collect():
                    done += self._finish(batch, recs, "", now)
                    progressed = True
            if progressed:
                continue
            if streamed and self.backend.inflight:
                # a launch is running: wake on a finished preparation, or
                # block until the oldest launch is over
                if futures:
                    cf.wait(list(futures), timeout=0.0002, return_when=cf.FIRST_COMPLETED)
                else:
                    self.backend.wait_oldest()
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


def _finish_batch(server, batch, recs, err, now):
    for i, st in enumerate(batch):
        if recs is None:
            st.status, st.error = "failed", err or "device step failed"
        else:
            st.records = recs[i]
            st.hr = decide_results(st.prep, recs[i])
            st.status = "done"
        st.t_done = now()
        server.used -= st.prep.footprint
        server.backend.release(st)
    return len(batch)


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
