"""Batched HR search: many jobs (functions, binades, sub-intervals of uneven
piece length) as work items of one persistent launch.

A job covers `count` consecutive binary64 arguments from X0.  It is cut
into sub-intervals of `sub_len` arguments (the last one shorter if needed),
each with its own piece length N (given per sub-interval, given once, or
chosen by the autotuner) and a partial last piece when N does not divide
the sub-interval.  The host makes one upper table per range of the job
(``plan.upper_ranges``) and the windows and thresholds of its
sub-intervals; the device makes every sub-interval's table from the upper
tables (hr_subtables) into one table pool; the pieces are split into work
items (``autotune.split_sub``).

Two forms run the same kernel on the same items:
  plain    one launch per job (one wave per item), results read back per job;
  batched  one persistent launch over every item of every job (grouped by
           word width and degree), items ordered by decreasing modelled cost.
Both give identical result sets.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib, api, autotune
from .plan import (BatchJob, PlannedJob, PlannedSub, TablePlan, job_items,  # noqa: F401
                   job_windows, plan_job, split_by_job, sub_costs, upper_ranges)
from .prep import JobSpec, is_hr

M64 = 1 << 64


@dataclass
class Plan:
    jobs: list                # PlannedJob, in job order
    tables: list              # (TablePlan, word offset of its table region in the pool)
    pool_words: int           # size of the device table pool
    items: np.ndarray         # api.ITEM_DTYPE, grouped by job then sub (plain order)
    variants: list            # (W, delta) of each item
    prep_s: float = 0.0

    def job_items(self, j: int):
        return np.nonzero(self.items["job"] == j)[0]


def build_plan(jobs, target_items: int = 16384, model=autotune.MODEL) -> Plan:
    """Plan every job (upper tables, windows) and split it into work items of
    about equal modelled cost over the whole batch."""
    t0 = time.time()
    staged = []
    total = 0.0
    for j in jobs:
        pj = plan_job(j)
        ranges = upper_ranges(pj)
        win, thr = job_windows(pj, ranges)
        total += sub_costs(pj, win, model)
        staged.append((pj, ranges, win, thr))
    target = max(total / target_items, 1e-9)
    tables, item_parts, variants = [], [], []
    base = 0
    for pj, ranges, win, thr in staged:
        items = job_items(pj, win, thr, target, model)
        tp = TablePlan(pj.job, pj.delta, pj.W, str(pj.uf),
                       [(sp.start, sp.length, sp.N) for sp in pj.subs],
                       [(lo, hi, U.Du, U.Wu, U.words) for lo, hi, U in ranges],
                       np.array([sp.N for sp in pj.subs], np.uint32), win, thr, items)
        tables.append((tp, base))
        items = items.copy()
        items["table"] += base
        item_parts.append(items)
        variants += [(pj.W, pj.delta)] * len(items)
        base += tp.table_words
    items = np.concatenate(item_parts) if item_parts else np.zeros(0, api.ITEM_DTYPE)
    return Plan([s[0] for s in staged], tables, max(base, 1), items, variants, time.time() - t0)


def make_tables(ctx, pool, base: int, tp: TablePlan, stream=None):
    """Launch hr_subtables for every range of one job: its sub-interval tables
    into pool[base:] (words), on the device."""
    E = tp.entries
    L = tp.W // 64
    for lo, hi, Du, Wu, words in tp.ranges:
        upper = api.to_dev(words.reshape(-1), torch.uint64, pool.device)
        Ns = api.to_dev(tp.Ns[lo:hi], torch.uint32, pool.device)
        out = pool[base + lo * E * L: base + hi * E * L]
        _lib.hr_subtables(ctx, upper, Du, Wu, None, 0, Ns, 0, hi - lo - 1, int(tp.Ns[lo:hi].max()),
                          hi - lo, tp.delta, tp.W, out, stream)


class DevicePlan:
    """A plan resident in HBM: the table pool (made on the device from the
    upper tables) and the items (plain and cost-sorted orders)."""

    def __init__(self, plan: Plan, model=autotune.MODEL, device="cuda", ctx=None):
        self.plan = plan
        ctx = ctx or api.context()
        self.pool = torch.empty(plan.pool_words, dtype=torch.uint64, device=device)
        ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        ev[0].record()
        for tp, base in plan.tables:
            make_tables(ctx, self.pool, base, tp)
        ev[1].record()
        torch.cuda.synchronize()
        self.tables_ms = ev[0].elapsed_time(ev[1])
        raw = plan.items.view(np.uint8).reshape(-1)
        self.items = api.to_dev(raw, torch.uint8, device)
        # batched order: by variant, then decreasing modelled cost
        cost = np.array([model.cost(it["npieces"], int(it["N"]),
                                    float(it["win_d"]) / 2.0 ** 64 * int(it["npieces"]) * int(it["N"]))
                         for it in plan.items])
        var = np.array([v[0] * 16 + v[1] for v in plan.variants])
        order = np.lexsort((-cost, var))
        self.sorted_items = api.to_dev(plan.items[order].view(np.uint8).reshape(-1), torch.uint8, device)
        self.groups = []          # (W, delta, first, count) over sorted_items
        vs = var[order]
        i = 0
        while i < len(vs):
            j = i
            while j < len(vs) and vs[j] == vs[i]:
                j += 1
            W, d = plan.variants[order[i]]
            self.groups.append((W, d, i, j - i))
            i = j
        self.job_groups = []      # per job: (W, delta, first, count) over plain items
        for j, pj in enumerate(plan.jobs):
            idx = plan.job_items(pj.job.job_id)
            self.job_groups.append((pj.W, pj.delta, int(idx[0]), len(idx)) if len(idx) else None)


def _run(ctx, dp, items_t, first, count_items, W, delta, waves, out, cap, count, stats, stream):
    base = items_t[first * _lib.ITEM_BYTES:(first + count_items) * _lib.ITEM_BYTES]
    _lib.hr_batch_run(ctx, dp.pool, base, count_items, W, delta, waves, out, cap, count, stats,
                      stream)


def device_waves() -> int:
    """Persistent grid size: every wave the device keeps resident (the
    library queries the kernel's occupancy)."""
    return _lib.HR_WAVES_FILL


class Runner:
    """Owns output buffers; runs a DevicePlan in plain or batched form."""

    def __init__(self, dp: DevicePlan, cap: int = 1 << 20, ctx=None):
        self.dp = dp
        self.ctx = ctx or api.context()
        self.cap = cap
        dev = dp.pool.device
        self.out = torch.empty(cap * _lib.RESULT_BYTES, dtype=torch.uint8, device=dev)
        self.count = torch.zeros(1, dtype=torch.uint64, device=dev)
        self.stats = torch.zeros(8, dtype=torch.uint64, device=dev)

    def _results(self):
        n = api._u64_scalar(self.count)
        if n > self.cap:
            raise _lib.HRError("hr_batch_run", _lib.HR_ECAPACITY)
        return self.out[: n * _lib.RESULT_BYTES].cpu().numpy().view(api.RESULT_DTYPE).copy()

    def _grow(self, n):
        self.cap = 1 << (n - 1).bit_length()
        self.out = torch.empty(self.cap * _lib.RESULT_BYTES, dtype=torch.uint8,
                               device=self.dp.pool.device)

    def batched(self, waves: int | None = None, stream=None, sync=True):
        """One persistent launch per (W, delta) group of the whole plan."""
        waves = waves or device_waves()
        while True:
            self.count.zero_()
            self.stats.zero_()
            for W, d, first, n in self.dp.groups:
                _run(self.ctx, self.dp, self.dp.sorted_items, first, n, W, d, waves, self.out,
                     self.cap, self.count, self.stats, stream)
            if not sync:
                return None
            torch.cuda.synchronize()
            n = api._u64_scalar(self.count)
            if n <= self.cap:
                return self._results()
            self._grow(n)

    def plain(self, stream=None):
        """One launch per job, each read back before the next one starts."""
        self.stats.zero_()
        parts = []
        for g in self.dp.job_groups:
            if g is None:
                continue
            W, d, first, n_items = g
            before = self.stats.clone()
            while True:
                self.count.zero_()
                self.stats.copy_(before)
                _run(self.ctx, self.dp, self.dp.items, first, n_items, W, d, 0, self.out,
                     self.cap, self.count, self.stats, stream)
                torch.cuda.synchronize()
                n = api._u64_scalar(self.count)
                if n <= self.cap:
                    break
                self._grow(n)
            parts.append(self._results())
        return np.concatenate(parts) if parts else np.zeros(0, api.RESULT_DTYPE)

    def capture(self, waves: int | None = None, cap: int | None = None):
        """Capture the batched launch sequence (counter fills + one persistent
        launch per group) in a HIP graph; returns a GraphRun with its own
        fixed-size output buffers (results beyond `cap` raise on read).
        Counters are cleared by fill kernels inside the graph, never by
        memset nodes."""
        waves = waves or device_waves()
        cap = cap or self.cap
        dev = self.dp.pool.device
        out = torch.empty(cap * _lib.RESULT_BYTES, dtype=torch.uint8, device=dev)
        count = torch.zeros(1, dtype=torch.uint64, device=dev)
        stats = torch.zeros(8, dtype=torch.uint64, device=dev)

        def launches(stream):
            count.zero_()
            stats.zero_()
            for W, d, first, n in self.dp.groups:
                _run(self.ctx, self.dp, self.dp.sorted_items, first, n, W, d, waves, out, cap,
                     count, stats, stream)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):        # warm up: context scratch exists
            launches(None)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            launches(None)
        return GraphRun(g, out, count, stats, cap)

    def stats_dict(self):
        st = self.stats.cpu().numpy()
        return {"pieces": int(st[0]), "candidates": int(st[1]), "results": int(st[2]),
                "partial_quotients": int(st[3]), "full_evaluations": int(st[5]),
                "nmdm": 1.0 - int(st[3]) / int(st[4]) if int(st[4]) else 0.0}


class GraphRun:
    """A captured batched pass: replay() relaunches it, results() reads it."""

    def __init__(self, graph, out, count, stats, cap):
        self.graph, self.out, self.count, self.stats, self.cap = graph, out, count, stats, cap

    def replay(self):
        self.graph.replay()

    def results(self):
        torch.cuda.synchronize()
        n = api._u64_scalar(self.count)
        if n > self.cap:
            raise _lib.HRError("hr_batch_run", _lib.HR_ECAPACITY)
        return self.out[: n * _lib.RESULT_BYTES].cpu().numpy().view(api.RESULT_DTYPE).copy()


def finish(plan: Plan, results: np.ndarray):
    """Per-job sorted HR offsets (argument X0 + m h), undecided values
    decided at high precision on the host."""
    out = {}
    per_job = split_by_job(results, [pj.job.job_id for pj in plan.jobs])
    for pj, res in zip(plan.jobs, per_job):
        jid = pj.job.job_id
        starts = np.array([sp.start for sp in pj.subs], dtype=np.int64)
        Ns = np.array([sp.N for sp in pj.subs], dtype=np.int64)
        sub = res["sub"].astype(np.int64)
        m = starts[sub] + res["piece"].astype(np.int64) * Ns[sub] + res["k"].astype(np.int64)
        hr = m[res["cls"] == 1].tolist()
        und = m[res["cls"] == 2].tolist()
        if und:
            spec = JobSpec(pj.job.fname, pj.job.X0, pj.job.count, pj.job.s, pj.job.mode)
            hr += [x for x in und if is_hr(spec, x, pj.uf)]
        out[jid] = sorted(hr)
    return out


def args_of(plan: Plan) -> int:
    return sum(pj.job.count for pj in plan.jobs)
