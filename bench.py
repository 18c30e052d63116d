"""Benchmark: binary64 arguments checked per second on the 2^40-argument exp
slice (exp on [1, 1 + 2^-12), round-to-nearest, eps = 2^-32 ulp; 4096
sub-intervals of 2^28 arguments, degree-4 tables at 256 bits, degree-1 pieces
of N = 2^18).

One step is one pass of the whole hot path over the slice with the range's
upper table (a degree-7 polynomial at 256 bits, 1.15 KB) resident in HBM: the
4096 sub-interval tables made on the device, tabulation of the 2^22 pieces,
degree-1 search of every piece, exact recheck of every candidate (the last
three fused in one launch), and the result list copied back to the host.
Beside it: the plain launch chain (tabulate -> search -> recheck) on the
same tables, the tabulation stage alone against a plain fill of the same
bytes, the plain search workload and the small pipeline, a stream of
distinct jobs end to end (host preparation included), the slice with its
pieces split 2 and 4 ways, the paper's lower-bound tests, the CPU SIMD
search, the batched mix (with its kernel's algorithmic VALU fraction), the
hard binade and the serving loop.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "binary64 args checked/sec (exp, 2^40 slice); batched vs plain speedup, p99"
PEAK_INT32_OPS = 256 * 64 * 2.4e9     # 256 CUs x 64 lanes x 2.4 GHz, one op/lane/clock
PEAK_HBM = 8.0e12                     # bytes/s

# HBM bytes per launch measured by rocprofv3 (FETCH_SIZE x 2.000 and
# WRITE_SIZE x 1.000, the factors a 1 GiB copy gives; summary under
# profiles/), valid only for the kernel sources they were taken on.
PROFILED_SOURCES = "40ed1c3e663831aa"      # sha256 prefix of hr_lib.hip + hr_core.h
PROFILED_TRAFFIC = {"k_pipeline<8,4>": 5.01e6, "k_tabulate<8,4>": 68.96e6}


def profiled_traffic(kernel):
    import hashlib
    csrc = os.path.join(ROOT, "paper_1211_3056_amd", "csrc")
    h = hashlib.sha256()
    for f in ("hr_lib.hip", "hr_core.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return PROFILED_TRAFFIC.get(kernel) if h.hexdigest()[:16] == PROFILED_SOURCES else None


# The paper's own figures (Sec. 6, Tables 5-6): whole computation (tabulation
# + search) of exp on binary64 [1, 2), Fermi C2070 + Xeon X5650 against the
# same Xeon: context, not a target.
PAPER_CONTEXT = {
    "speedup_vs_1_core": 53.4, "speedup_vs_6_cores_12_ranks": 7.1,
    "hardware": "NVIDIA Tesla C2070 (Fermi, 14 SMs) + Intel Xeon X5650 (6 cores, 2.67 GHz)",
    "workload": "exp, binary64 binade [1, 2), directed (53, 2^-32) HR cases",
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--cpu-subs", type=int, default=16,
                   help="sub-intervals in the oracle's timed sample")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain workload")
    p.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    p.add_argument("--serve-jobs", type=int, default=2000)
    p.add_argument("--prep-workers", type=int, default=16)
    p.add_argument("--probe", action="store_true",
                   help="profiling probe: a 1 GiB device copy, then 3 fused passes of the "
                        "2^40 slice, 3 tabulations of it and 3 batched passes of the 16-job "
                        "mix; no JSON")
    return p.parse_args()


def ops_model(spec, pieces, cand, quotients, full):
    """Algorithmic int32 VALU operations of one pass:
    tabulation: one 32-bit limb add per limb of each difference-row update,
    sum_j (delta - j) W/32 per piece; search: 96 ops per partial quotient of
    the exact closest-point walk plus 12 per candidate step; recheck: each
    candidate multiplies delta words of the top 128 bits of its rows by a
    128-bit binomial (4 x 4 limb products truncated to 128 bits, 2 ops each)
    and adds them; the `full` candidates not rejected that way repeat it at
    the full W bits."""
    L = spec.W // 32

    def rechk(limbs):
        mul = 2 * sum(max(limbs - j, 0) for j in range(4))
        return spec.delta * (mul + limbs) + 12

    tab = sum(spec.delta - j for j in range(spec.delta + 1)) * L
    top = rechk(4) if L > 4 else 0
    return pieces * tab + quotients * 96 + cand * top + full * rechk(L)


class FusedStep:
    """One pass of the hot path over a resident job: the sub-interval tables
    made on the device from the range's upper table (hr_subtables), then the
    fused tabulate + search + recheck (hr_pipeline), then the result rows
    copied back.  HIP events bracket the two launches on their stream."""

    def __init__(self, spec, ctx, stream, Du=None, Wu=None, cap=1 << 16):
        import torch

        from paper_1211_3056_amd import _lib, autotune, pipeline
        self.spec, self.ctx, self.stream, self.cap = spec, ctx, stream, cap

        def prepare(sp):
            du = Du or autotune.choose_upper_degree(sp.fname, sp.X0, sp.count, sp.s, sp.delta)
            wu = Wu or autotune.choose_upper_width(du, sp.n_sub, sp.N, sp.tau, sp.delta, sp.s)
            return pipeline.UpperPrepared(sp, du, wu)

        # host preparation (degree and width choice, upper table, window and
        # thresholds): the first job of the process builds the integer
        # matrices shared by every job of this shape; the next slice of the
        # same function shows what a new job costs after that
        t0 = time.perf_counter()
        self.Pu = prepare(spec)
        self.prep_cold_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        prepare(dataclasses.replace(spec, X0=spec.X0 + spec.count * 2.0 ** -52))
        self.prep_s = time.perf_counter() - t0
        self.upper, self.win, self.thr = pipeline.upload_upper(self.Pu)
        dev = self.upper.device
        E = (spec.delta + 1) * (spec.delta + 2) // 2
        self.table = torch.empty(spec.n_sub * E * (spec.W // 64), dtype=torch.uint64, device=dev)
        self.RB = _lib.RESULT_BYTES
        # one device buffer: count, stats[8], padding to 96 bytes, then the
        # result rows, so that a step copies its outputs back in one transfer
        H = 12
        self.H = H
        self.dev = torch.zeros(H + cap * self.RB // 8, dtype=torch.uint64, device=dev)
        self.counters = self.dev[:9]
        self.count, self.stats = self.dev[:1], self.dev[1:9]
        self.out = self.dev[H:].view(torch.uint8)
        self.host = torch.zeros(H + cap * self.RB // 8, dtype=torch.uint64).pin_memory()
        self.count_h = self.host[:1]
        self.res_h = self.host[H:].view(torch.uint8)
        # rows fetched per step: every step searches the same batch, so the
        # last count (rounded up) bounds this one; rows beyond it are fetched
        # after the loop, inside the timed region
        self.fetch = cap

    def __call__(self, ev=None):
        import torch

        from paper_1211_3056_amd import _lib, pipeline
        sp, st = self.spec, self.stream
        # the clearing and the copy back go on the step's stream, ordered
        # with its launches
        with torch.cuda.stream(st):
            self.counters.zero_()
            if ev:
                ev[0].record(st)
            pipeline.make_tables(self.Pu, self.upper, ctx=self.ctx, stream=st, out=self.table)
            if ev:
                ev[1].record(st)
            _lib.hr_pipeline(self.ctx, self.table, sp.n_sub, sp.delta, sp.tau, sp.W, sp.N,
                             self.win, self.thr, self.out, self.cap, self.count, self.stats, st)
            if ev:
                ev[2].record(st)
            n = self.H + self.fetch * self.RB // 8
            self.host[:n].copy_(self.dev[:n], non_blocking=True)

    def settle(self):
        """After warm-up: fetch only the rows the last pass produced."""
        self.fetch = min(self.cap, -(-max(int(self.count_h.numpy()[0]), 1) // 1024) * 1024)

    def finish(self):
        """Rows beyond the prefix (none while every step repeats one batch);
        returns (result records, stats array)."""
        from paper_1211_3056_amd import api
        n_res = int(self.count_h.numpy()[0])
        assert n_res <= self.cap
        if self.fetch < n_res:
            self.res_h[self.fetch * self.RB: n_res * self.RB].copy_(
                self.out[self.fetch * self.RB: n_res * self.RB])
        res = self.res_h[: n_res * self.RB].numpy().view(api.RESULT_DTYPE)
        return res, self.stats.cpu().numpy()


def timed_steps(step, steps, warmup):
    """(wall ms per step, [(tables ms, pipeline ms)] per step by HIP events)."""
    import torch
    for _ in range(warmup):
        step()
        torch.cuda.synchronize()
        step.settle()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    res, st = step.finish()
    wall = time.perf_counter() - t0
    return wall * 1000 / steps, [(a.elapsed_time(b), b.elapsed_time(c)) for a, b, c in evs], res, st


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the search "
              "shards by sub-interval with no communication, and that split is a design, "
              "not a measured path", file=sys.stderr)
        sys.exit(2)
    pool = None
    if args.probe:
        args.no_serve = True
    else:
        # preparation workers come from a forkserver started before the GPU is used
        from paper_1211_3056_amd import serve
        pool = serve.make_pool(args.prep_workers)
    import torch

    import synth
    from paper_1211_3056_amd import api, pipeline
    from paper_1211_3056_amd.prep import JobSpec

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe:
        probe()
        return
    spec = JobSpec(**synth.CONFIG3)
    ctx = api.context()
    stream = torch.cuda.current_stream()
    step = FusedStep(spec, ctx, stream)
    ms_per_step, ev_ms, res, st = timed_steps(step, args.steps, args.warmup)
    tab_ms = [a for a, _ in ev_ms]
    kern_ms = [b for _, b in ev_ms]
    pieces, cand, quot, full = int(st[0]), int(st[1]), int(st[3]), int(st[5])
    hr_cases = int((res["cls"] == 1).sum())
    undecided = int((res["cls"] == 2).sum())
    args_total = spec.count
    value = args_total / (ms_per_step / 1000)
    kern_avg = sum(kern_ms) / len(kern_ms)
    ops = ops_model(spec, pieces, cand, quot, full)
    achieved = ops / (kern_avg / 1000) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "args/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "exp_rn_slice_2^40_[1,1+2^-12)_eps2^-32_N2^18_tau2^10_deg4_W256",
                   "form": "fused, sub-interval tables made on the device",
                   "sub_intervals": spec.n_sub, "pieces": pieces,
                   "upper_degree": step.Pu.Du, "upper_width": step.Pu.Wu},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32 VALU, algorithmic)",
                     "frac": achieved / (PEAK_INT32_OPS / 1e12),
                     "traffic": profiled_traffic("k_pipeline<8,4>"),
                     "kernel": "k_pipeline<8,4>", "kernel_ms": kern_avg,
                     "kernel_ms_median": sorted(kern_ms)[len(kern_ms) // 2]},
        "subtables_ms": sum(tab_ms) / len(tab_ms),
        "hr_cases": hr_cases, "undecided": undecided, "candidates": cand,
        "full_width_evaluations": full,
        "partial_quotients": quot, "quotients_per_piece": quot / max(pieces, 1),
        "nmdm_wave64": 1.0 - quot / int(st[4]) if int(st[4]) else 0.0,
        "host_prep_s": step.prep_s,
        "host_prep_first_job_s": step.prep_cold_s,
        "end_to_end_args_per_s": args_total / (step.prep_s + ms_per_step / 1000),
        "end_to_end_first_job_args_per_s": args_total / (step.prep_cold_s + ms_per_step / 1000),
    }
    line["end_to_end_stream"] = bench_stream(spec, ctx, stream)
    line["tabulation"] = bench_tabulation(spec, step.table, ctx, stream, args.steps)
    line["config1"] = bench_config1(ctx, stream, args.steps)
    line["config2"] = bench_config2(ctx, stream, args)
    line["refinement"] = bench_refinement(spec, ctx, stream, res)
    line["filters"] = bench_filters(ctx, stream)
    line["cpu_simd"] = bench_cpu_simd(step, ctx, stream)
    if not args.no_plain:
        line["plain_form"] = bench_plain(step, ctx, stream)
    if not args.no_batch:
        line["batch"] = bench_batch(args)
        line["hard_binade"] = bench_hard_binade(args)
    if not args.no_serve:
        line["serving"] = bench_serve(args, pool)
    line["paper_context"] = dict(PAPER_CONTEXT)
    if not args.no_cpu_baseline:
        from oracle import hr as ohr
        from oracle import native
        from oracle.taylor import Job
        job = Job(**synth.CONFIG3)
        n_sub = spec.n_sub
        subs = list(range(0, n_sub, max(1, n_sub // args.cpu_subs)))[: args.cpu_subs]
        t0 = time.perf_counter()
        ohr.pipeline(job, subs=subs)
        cpu_s = time.perf_counter() - t0
        one = subs[: max(1, len(subs) // 8)]           # a smaller sample on one thread
        t0 = time.perf_counter()
        ohr.pipeline(job, subs=one, threads=1)
        one_s = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(subs) * spec.per_sub / cpu_s, "unit": "args/s",
                                "cores": native.threads_default(), "kind": "oracle",
                                "sample": f"{len(subs)} of {n_sub} sub-intervals "
                                          f"({len(subs) * spec.per_sub} args), {cpu_s:.1f} s",
                                "value_1_thread": len(one) * spec.per_sub / one_s,
                                "sample_1_thread": f"{len(one)} sub-intervals, {one_s:.1f} s",
                                "nproc": os.cpu_count(), "cpu_model": cpu_model(),
                                "gpu_over_cpu": value / (len(subs) * spec.per_sub / cpu_s)}
    print(json.dumps(line))


def bench_stream(spec, ctx, stream, n_jobs=8):
    """End to end over a stream of distinct jobs: n_jobs consecutive 2^40
    slices of exp (X0 = 1 + i 2^-12), each prepared on the host (degree and
    width of its upper polynomial, upper table, window, thresholds), made
    into tables and searched on the device,
    and finished on the host (undecided values decided at high precision).
    The host preparation of the next job overlaps the device pass of the
    current one."""
    import torch

    from paper_1211_3056_amd import _lib, api, autotune, pipeline
    specs = [dataclasses.replace(spec, X0=1.0 + i * 2.0 ** -12) for i in range(n_jobs)]
    RB = _lib.RESULT_BYTES
    cap = 1 << 16
    E = (spec.delta + 1) * (spec.delta + 2) // 2
    bufs = []
    for _ in range(2):
        bufs.append({"table": torch.empty(spec.n_sub * E * (spec.W // 64), dtype=torch.uint64,
                                          device="cuda"),
                     "out": torch.empty(cap * RB, dtype=torch.uint8, device="cuda"),
                     "count": torch.zeros(1, dtype=torch.uint64, device="cuda"),
                     "count_h": torch.zeros(1, dtype=torch.uint64).pin_memory(),
                     "res_h": torch.zeros(cap * RB, dtype=torch.uint8).pin_memory(),
                     "done": torch.cuda.Event()})

    def launch(Pu, b):
        with torch.cuda.stream(stream):
            upper, win, thr = pipeline.upload_upper(Pu)
            pipeline.make_tables(Pu, upper, ctx=ctx, stream=stream, out=b["table"])
            b["count"].zero_()
            sp = Pu.spec
            _lib.hr_pipeline(ctx, b["table"], sp.n_sub, sp.delta, sp.tau, sp.W, sp.N, win, thr,
                             b["out"], cap, b["count"], None, stream)
            b["count_h"].copy_(b["count"], non_blocking=True)
            b["res_h"].copy_(b["out"], non_blocking=True)
            b["done"].record(stream)

    def finish(Pu, b):
        b["done"].synchronize()
        n = int(b["count_h"].numpy()[0])
        assert n <= cap
        res = b["res_h"][: n * RB].numpy().view(api.RESULT_DTYPE)
        hr, _ = pipeline._finish(Pu, res["sub"], res["piece"], res["k"], res["cls"])
        return len(hr)

    # one untimed job through both buffer sets first (a slice after the
    # measured ones): pinned staging buffers and the launch path are warm
    for i in range(2):
        sp = dataclasses.replace(spec, X0=1.0 + (n_jobs + i) * 2.0 ** -12)
        Du = autotune.choose_upper_degree(sp.fname, sp.X0, sp.count, sp.s, sp.delta)
        Wu = autotune.choose_upper_width(Du, sp.n_sub, sp.N, sp.tau, sp.delta, sp.s)
        Pw = pipeline.UpperPrepared(sp, Du, Wu)
        launch(Pw, bufs[i])
        finish(Pw, bufs[i])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prep_s = 0.0
    pending = None
    cases = 0
    for i, sp in enumerate(specs):
        t1 = time.perf_counter()
        Du = autotune.choose_upper_degree(sp.fname, sp.X0, sp.count, sp.s, sp.delta)
        Wu = autotune.choose_upper_width(Du, sp.n_sub, sp.N, sp.tau, sp.delta, sp.s)
        Pu = pipeline.UpperPrepared(sp, Du, Wu)
        prep_s += time.perf_counter() - t1
        b = bufs[i % 2]
        launch(Pu, b)
        if pending:
            cases += finish(*pending)
        pending = (Pu, b)
    cases += finish(*pending)
    wall = time.perf_counter() - t0
    return {"jobs": n_jobs, "args": n_jobs * spec.count, "wall_s": wall,
            "args_per_s": n_jobs * spec.count / wall, "host_prep_s_per_job": prep_s / n_jobs,
            "hr_cases": cases,
            "workload": f"{n_jobs} consecutive 2^40 slices of exp from 1.0, eps 2^-32 RN"}


def bench_plain(step, ctx, stream, reps=3):
    """The plain launch chain on the same resident tables: hr_tabulate (a, b
    of every piece to HBM), hr_search (candidate list to HBM), hr_recheck.
    Device time by HIP events (the search's hit total is read on the host
    between the search and the recheck); wall time includes that read and
    the copy of the classes back."""
    import numpy as np
    import torch

    from paper_1211_3056_amd import _lib, api
    sp = step.spec
    n = sp.n_sub * sp.tau
    dev = step.table.device
    a = torch.empty(n, dtype=torch.uint64, device=dev)
    b = torch.empty(n, dtype=torch.uint64, device=dev)
    N = api.to_dev(np.full(n, sp.N, np.uint32), torch.uint32)
    w = step.win.view(-1, 2)
    lo, d = w[:, 0].contiguous(), w[:, 1].contiguous()
    width = int(step.Pu.win[1])
    cap = int(width / 2.0 ** 64 * sp.count * 1.25) + (1 << 16)
    counts = torch.empty(n, dtype=torch.uint32, device=dev)
    offsets = torch.empty(n, dtype=torch.uint64, device=dev)
    hits = torch.empty(cap, dtype=torch.uint32, device=dev)
    inst = torch.empty(cap, dtype=torch.uint32, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    value = torch.empty(cap, dtype=torch.uint64, device=dev)
    cls = torch.empty(cap, dtype=torch.uint8, device=dev)
    best = None
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record(stream)
        _lib.hr_tabulate(ctx, step.table, sp.n_sub, sp.delta, sp.tau, sp.W, a, b, stream)
        _lib.hr_search(ctx, a, b, N, lo, d, sp.tau, counts, offsets, hits, inst, cap, total,
                       stream)
        ev[1].record(stream)
        n_cand = int(total.cpu().numpy()[0])
        assert n_cand <= cap
        ev[2].record(stream)
        _lib.hr_recheck(ctx, step.table, sp.n_sub, sp.delta, sp.tau, sp.W, inst[:n_cand],
                        hits[:n_cand], sp.N - 1, step.thr, value, cls, stream)
        ev[3].record(stream)
        cls_h = cls[:n_cand].cpu().numpy()
        wall = time.perf_counter() - t0
        dev_ms = ev[0].elapsed_time(ev[1]) + ev[2].elapsed_time(ev[3])
        if best is None or dev_ms < best[0]:
            best = (dev_ms, wall, n_cand, int((cls_h == 1).sum()))
    dev_ms, wall, n_cand, n_hr = best
    return {"device_ms": dev_ms, "wall_ms": wall * 1000, "value": sp.count / (dev_ms / 1000),
            "candidates": n_cand, "hr_cases": n_hr,
            "launches": "hr_tabulate, hr_search (3 kernels), hr_recheck"}


def wave_stats(it, width):
    """min / max / mean of per-instance loop passes, and the mean over groups
    of `width` consecutive lanes of the idle fraction 1 - sum / (width max)
    (the paper's NMDM, Sec. 2.2)."""
    import numpy as np
    it = it.astype(np.float64)
    g = it[: len(it) // width * width].reshape(-1, width)
    mx = g.max(axis=1)
    nmdm = np.where(mx > 0, 1.0 - g.mean(axis=1) / np.maximum(mx, 1), 0.0)
    return {"min": int(it.min()), "max": int(it.max()), "mean": float(it.mean()),
            "nmdm": float(nmdm.mean())}


def bench_filters(ctx, stream, reps=5):
    """The paper's lower-bound tests against the exact walk on the Table 3
    workload's pieces: exp on [1, 1 + 2^-13) (2^39 arguments, directed,
    eps = 2^-32, pieces of N = 2^15, degree 3 at 192 bits; 2^24 pieces,
    tables made on the device).  Per test: kernel time (HIP events), loop
    passes per piece (min / max / mean) and the idle fraction of a 64-lane
    wave and of a 32-lane group (the paper's warp), and the share of pieces
    it certifies.  The exact walk's partial quotients come from
    hr_search_steps, its time from hr_search over the same pieces."""
    import numpy as np
    import torch

    from paper_1211_3056_amd import _lib, api, autotune, pipeline
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec("exp", 1.0, 1 << 39, 32, "dir", 1 << 15, 1 << 13, 3, 192)
    Du = autotune.choose_upper_degree(spec.fname, spec.X0, spec.count, spec.s, spec.delta)
    Wu = autotune.choose_upper_width(Du, spec.n_sub, spec.N, spec.tau, spec.delta, spec.s)
    P = pipeline.UpperPrepared(spec, Du, Wu)
    upper, win, thr = pipeline.upload_upper(P)
    table = pipeline.make_tables(P, upper, ctx=ctx, stream=stream)
    a, b = api.tabulate(table, spec.n_sub, spec.delta, spec.tau, spec.W, ctx=ctx, stream=stream)
    n = a.numel()
    N = api.to_dev(np.full(n, spec.N, np.uint32), torch.uint32)
    lo = api.to_dev(np.full(1, P.win[0], np.uint64), torch.uint64)
    d = api.to_dev(np.full(1, P.win[1], np.uint64), torch.uint64)
    passed = torch.empty(n, dtype=torch.uint8, device="cuda")
    iters = torch.empty(n, dtype=torch.uint32, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        return min(e0.elapsed_time(e1) for e0, e1 in evs)

    out = {"workload": "exp dir [1,1+2^-13) 2^39 args, eps 2^-32, N = 2^15: 2^24 pieces",
           "pieces": n}
    for name, alg in (("lefevre_alg3", _lib.HR_FILTER_LEFEVRE),
                      ("regular_alg4", _lib.HR_FILTER_REGULAR)):
        ms = timed(lambda: _lib.hr_filter(ctx, alg, a, b, N, lo, d, n, passed, None, iters,
                                          stream))
        it = iters.cpu().numpy()
        w64, w32 = wave_stats(it, 64), wave_stats(it, 32)
        out[name] = {"kernel_ms": ms, "iters_min": w64["min"], "iters_max": w64["max"],
                     "iters_mean": w64["mean"], "nmdm_wave64": w64["nmdm"],
                     "nmdm_32_lanes": w32["nmdm"],
                     "certified_frac": float(passed.cpu().numpy().mean())}
    steps = torch.empty(n, dtype=torch.uint32, device="cuda")
    _lib.hr_search_steps(ctx, a, b, N, lo, d, n, steps, stream)
    st = steps.cpu().numpy()
    counts = torch.empty(n, dtype=torch.uint32, device="cuda")
    offsets = torch.empty(n, dtype=torch.uint64, device="cuda")
    cap = 1 << 24
    hits = torch.empty(cap, dtype=torch.uint32, device="cuda")
    total = torch.zeros(1, dtype=torch.uint64, device="cuda")
    ms = timed(lambda: _lib.hr_search(ctx, a, b, N, lo, d, n, counts, offsets, hits, None, cap,
                                      total, stream))
    w64, w32 = wave_stats(st, 64), wave_stats(st, 32)
    out["exact_walk"] = {"kernel_ms": ms, "quotients_min": w64["min"], "quotients_max": w64["max"],
                         "quotients_mean": w64["mean"], "nmdm_wave64": w64["nmdm"],
                         "nmdm_32_lanes": w32["nmdm"],
                         "pieces_without_candidates_frac": float(
                             (counts.cpu().numpy() == 0).mean()),
                         "candidates": int(total.cpu().numpy()[0])}
    out["paper_table4"] = {"lefevre": {"min": 5, "max": 328, "mean": 24, "nmdm": 0.256},
                           "lefevre_specific_instructions": {"min": 5, "max": 31, "mean": 16,
                                                             "nmdm": 0.257},
                           "regular": {"min": 8, "max": 19, "mean": 12, "nmdm": 0.001},
                           "hardware": "Fermi C2070, 32-thread warps"}
    return out


def bench_cpu_simd(step, ctx, stream):
    """The multi-core SIMD CPU search (libhrcpu.so: AVX-512 regular test,
    exact walk for the instances it does not certify) on the host cores,
    over the same 2^22 pieces of the 2^40 slice (tabulated on the device and
    copied to the host) and over the plain search workload; a stronger CPU
    comparison than the oracle, which is not tuned."""
    import numpy as np
    import torch

    import synth
    from paper_1211_3056_amd import _cpu, _lib
    sp = step.spec
    n = sp.n_sub * sp.tau
    a = torch.empty(n, dtype=torch.uint64, device="cuda")
    b = torch.empty(n, dtype=torch.uint64, device="cuda")
    _lib.hr_tabulate(ctx, step.table, sp.n_sub, sp.delta, sp.tau, sp.W, a, b, stream)
    torch.cuda.synchronize()
    A, B = a.cpu().numpy(), b.cpu().numpy()
    N = np.full(n, sp.N, np.uint32)
    lo, d = int(step.Pu.win[0]), int(step.Pu.win[1])
    t0 = time.perf_counter()
    counts, _, hits = _cpu.search(A, B, N, d, lo=lo, cap=1 << 25)
    t = time.perf_counter() - t0
    A1, B1, N1, D1 = synth.config1()
    t1 = time.perf_counter()
    c1, _, h1 = _cpu.search(A1, B1, N1, D1)
    t1 = time.perf_counter() - t1
    return {"simd_width": _cpu.simd_width(), "threads": os.cpu_count(),
            "slice_2^40_search_s": t, "slice_2^40_args_per_s": sp.count / t,
            "slice_2^40_candidates": int(len(hits)),
            "config1_s": t1, "config1_args_per_s": len(A1) * int(N1[0]) / t1,
            "config1_hits": int(len(h1)),
            "note": "degree-1 search only (tabulation and recheck not included)"}


def bench_refinement(spec, ctx, stream, res_ref):
    """The 2^40 slice with pieces split s ways from the start (N / s
    arguments, tau s pieces per sub-interval; the paper's phase-2 split
    applied to every piece): candidates fall about s^2-fold, the walks grow
    s-fold.  Same HR cases as the headline step, compared here."""
    import numpy as np
    out = {"workload": "config 3 with pieces of N/s arguments"}
    ref = np.sort(res_ref[res_ref["cls"] == 1], order=["sub", "piece", "k"])
    ref_m = (ref["sub"].astype(np.int64) * spec.per_sub + ref["piece"].astype(np.int64) * spec.N
             + ref["k"].astype(np.int64))
    for sdiv in (2, 4):
        sp = dataclasses.replace(spec, N=spec.N // sdiv, tau=spec.tau * sdiv)
        step = FusedStep(sp, ctx, stream)
        ms, ev_ms, res, st = timed_steps(step, 5, 2)
        hr = res[res["cls"] == 1]
        m = np.sort(hr["sub"].astype(np.int64) * sp.per_sub + hr["piece"].astype(np.int64) * sp.N
                    + hr["k"].astype(np.int64))
        out[f"s{sdiv}"] = {"N": sp.N, "ms_per_step": ms,
                           "kernel_ms": sum(b for _, b in ev_ms) / len(ev_ms),
                           "candidates": int(st[1]), "partial_quotients": int(st[3]),
                           "hr_cases": int(len(hr)),
                           "same_hr_as_headline": bool(np.array_equal(m, np.sort(ref_m)))}
    return out


def bench_hard_binade(args):
    """exp on 2^40 arguments of [128, 128 + 2^-5) (the hard binade of the
    paper's Tables 6 and 8: ulp(x) = 2^-45, so the degree-1 truncation over a
    piece is ~2^20 times larger than on [1, 2)), directed, eps = 2^-32, as a
    batched persistent launch over device-made tables (degree 5 at 128 bits,
    sub-intervals of 2^28).  With the paper's pieces of N = 2^15 a piece has
    about 100 candidates; the autotuner's shorter pieces (the refinement of
    the paper's phase 2 applied from the start, s = 2^15 / N sub-pieces per
    paper piece) cut the candidates by about s^2."""
    import torch

    from paper_1211_3056_amd import batch
    out = {"workload": "exp dir [128,128+2^-5) 2^40 args, eps 2^-32"}
    for name, N in (("paper_N_2^15", 1 << 15), ("autotuned", None)):
        job = batch.BatchJob("exp", 128.0, 1 << 40, 32, "dir", N=N, job_id=0)
        plan = batch.build_plan([job])
        dp = batch.DevicePlan(plan)
        run = batch.Runner(dp, cap=1 << 16)
        run.batched()
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            res = run.batched()
            ts.append(time.perf_counter() - t0)
        st = run.stats_dict()
        hr = batch.finish(plan, res)[0]
        pj = plan.jobs[0]
        out[name] = {"N": pj.subs[0].N, "delta": pj.delta, "W": pj.W,
                     "upper_degrees": sorted({r[2] for tp, _ in plan.tables for r in tp.ranges}),
                     "ms": min(ts) * 1000, "args_per_s": (1 << 40) / min(ts),
                     "candidates": st["candidates"], "hr_cases": len(hr),
                     "device_tables_ms": dp.tables_ms, "host_prep_s": plan.prep_s}
    out["refinement_factor"] = (1 << 15) // out["autotuned"]["N"]
    out["candidates_cut"] = out["paper_N_2^15"]["candidates"] / max(out["autotuned"]["candidates"], 1)
    return out


def bench_config1(ctx, stream, steps):
    """The plain degree-1 search alone: 4096 random (a, b), N = 2^16,
    threshold 2^-20 (hr_search's three launches, HIP events)."""
    import numpy as np
    import torch

    import synth
    from paper_1211_3056_amd import _lib, api
    A, B, N, D = synth.config1()
    a = api.to_dev(A, torch.uint64)
    b = api.to_dev(B, torch.uint64)
    Nd = api.to_dev(N, torch.uint32)
    d = api.to_dev(np.full(1, D, np.uint64), torch.uint64)
    n = len(A)
    counts = torch.empty(n, dtype=torch.uint32, device="cuda")
    offsets = torch.empty(n, dtype=torch.uint64, device="cuda")
    cap = 1 << 12
    hits = torch.empty(cap, dtype=torch.uint32, device="cuda")
    total = torch.zeros(1, dtype=torch.uint64, device="cuda")
    run = lambda: _lib.hr_search(ctx, a, b, Nd, None, d, n, counts, offsets, hits, None, cap,
                                 total, stream)
    run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for e0, e1 in evs:
        e0.record(stream)
        run()
        e1.record(stream)
    torch.cuda.synchronize()
    ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / steps
    stp = torch.empty(n, dtype=torch.uint32, device="cuda")
    _lib.hr_search_steps(ctx, a, b, Nd, None, d, n, stp, stream)
    quot = int(stp.to(torch.int64).sum().item())
    n_hits = int(total.cpu().numpy()[0])
    ops = quot * 96 + n_hits * 12
    return {"workload": "4096 random (a, b), N = 2^16, d = 2^-20", "kernel_ms": ms,
            "args_per_s": n * int(N[0]) / (ms / 1000), "hits": n_hits,
            "partial_quotients": quot,
            "roofline": {"bound": "alu", "achieved": ops / (ms / 1000) / 1e12,
                         "peak": PEAK_INT32_OPS / 1e12, "unit": "Tops/s (int32 VALU, algorithmic)",
                         "frac": ops / (ms / 1000) / PEAK_INT32_OPS,
                         "note": "4096 lanes fill 1/4 of one wave slot per SIMD: the "
                                 "workload is latency-bound by its size"}}


def bench_config2(ctx, stream, args):
    """exp on 2^32 arguments of [1, 1 + 2^-20) (256 sub-intervals, degree 3
    at 192 bits, N = 2^16, eps = 2^-24 RN): the same device-table + fused
    step as the headline."""
    import synth
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec(**synth.CONFIG2)
    step = FusedStep(spec, ctx, stream)
    ms, ev_ms, res, st = timed_steps(step, args.steps, args.warmup)
    kern = sum(b for _, b in ev_ms) / len(ev_ms)
    pieces, cand, quot, full = int(st[0]), int(st[1]), int(st[3]), int(st[5])
    ops = ops_model(spec, pieces, cand, quot, full)
    return {"workload": "exp_rn_[1,1+2^-20)_2^32args_eps2^-24_N2^16_tau2^8_deg3_W192",
            "ms_per_step": ms, "args_per_s": spec.count / (ms / 1000),
            "kernel": f"k_pipeline<{spec.W // 32},{spec.delta}>", "kernel_ms": kern,
            "subtables_ms": sum(a for a, _ in ev_ms) / len(ev_ms),
            "hr_cases": int((res["cls"] == 1).sum()), "candidates": cand,
            "host_prep_s": step.prep_s, "upper_degree": step.Pu.Du,
            "roofline": {"bound": "alu", "achieved": ops / (kern / 1000) / 1e12,
                         "peak": PEAK_INT32_OPS / 1e12, "unit": "Tops/s (int32 VALU, algorithmic)",
                         "frac": ops / (kern / 1000) / PEAK_INT32_OPS}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_tabulation(spec, table, ctx, stream, steps):
    """The tabulation stage alone (hr_tabulate: every piece's (a, b) of the
    2^40 slice written to HBM), timed with HIP events on its stream.
    Algorithmic bytes: the initial tables read once plus 16 bytes of (a, b)
    written per piece."""
    import torch

    from paper_1211_3056_amd import _lib
    pieces = spec.n_sub * spec.tau
    a_out = torch.empty(pieces, dtype=torch.uint64, device=table.device)
    b_out = torch.empty(pieces, dtype=torch.uint64, device=table.device)
    run = lambda: _lib.hr_tabulate(ctx, table, spec.n_sub, spec.delta, spec.tau, spec.W,
                                   a_out, b_out, stream)
    run()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        run()
        b.record(stream)
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    nbytes = table.numel() * 8 + pieces * 16
    kernel = f"k_tabulate<{spec.W // 32},{spec.delta}>"
    # achievable streaming-write rate: torch's fill of the same 16 bytes per
    # piece, timed the same way
    buf = torch.empty(2 * pieces, dtype=torch.int64, device=table.device)
    buf.fill_(1)
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        buf.fill_(3)
        b.record(stream)
    torch.cuda.synchronize()
    fill_ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    ceiling = pieces * 16 / (fill_ms / 1000)
    return {"kernel": kernel, "kernel_ms": ms, "pieces": pieces, "bytes": nbytes,
            "traffic": profiled_traffic(kernel), "hbm_GBps": nbytes / (ms / 1000) / 1e9,
            "hbm_frac": nbytes / (ms / 1000) / PEAK_HBM,
            "write_ceiling_GBps": ceiling / 1e9, "fill_ms": fill_ms,
            "ceiling_frac": nbytes / (ms / 1000) / ceiling,
            "pieces_per_s": pieces / (ms / 1000)}


def probe():
    """Kernels for counter runs: a plain copy of known size (the reference
    for scaling FETCH_SIZE / WRITE_SIZE), then three of each: the headline
    step (sub-interval tables from the upper table, fused pass), the
    tabulation stage, the batched pass of the 16-job mix, the plain search
    workload; one pass of each of the paper's tests over the 2^40 slice's
    pieces.  Progress on stderr."""
    import numpy as np
    import torch

    import synth
    from paper_1211_3056_amd import _lib, api, batch
    from paper_1211_3056_amd.prep import JobSpec

    def say(msg):
        print(f"probe: {msg}", file=sys.stderr, flush=True)

    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    say("copy done")
    ctx = api.context()
    stream = torch.cuda.current_stream()
    spec = JobSpec(**synth.CONFIG3)
    step = FusedStep(spec, ctx, stream)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    say("fused steps done")
    n = spec.n_sub * spec.tau
    a = torch.empty(n, dtype=torch.uint64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        _lib.hr_tabulate(ctx, step.table, spec.n_sub, spec.delta, spec.tau, spec.W, a, b, stream)
    torch.cuda.synchronize()
    say("tabulation done")
    N = api.to_dev(np.full(n, spec.N, np.uint32), torch.uint32)
    lo = api.to_dev(np.full(1, step.Pu.win[0], np.uint64), torch.uint64)
    d = api.to_dev(np.full(1, step.Pu.win[1], np.uint64), torch.uint64)
    passed = torch.empty(n, dtype=torch.uint8, device="cuda")
    for alg in (_lib.HR_FILTER_LEFEVRE, _lib.HR_FILTER_REGULAR):
        _lib.hr_filter(ctx, alg, a, b, N, lo, d, n, passed, None, None, stream)
    torch.cuda.synchronize()
    say("filters done")
    A, B, N1, D = synth.config1()
    for _ in range(3):
        api.search(api.to_dev(A, torch.uint64), api.to_dev(B, torch.uint64),
                   api.to_dev(N1, torch.uint32), D, ctx=ctx)
    say("plain search done")
    dp = batch.DevicePlan(batch.build_plan([batch.BatchJob(**d) for d in synth.config4()]))
    run = batch.Runner(dp)
    for _ in range(3):
        run.batched()
    torch.cuda.synchronize()
    say("batched passes done")


def bench_batch(args):
    """16 jobs (exp, log, 2^x, sin; 2^30..2^38 arguments each; N uniform in
    [2^12, 2^20] per sub-interval; eps = 2^-28): one persistent launch vs one
    launch per job, same work items, same results."""
    import numpy as np
    import torch

    import synth
    from paper_1211_3056_amd import batch

    jobs = [batch.BatchJob(**d) for d in synth.config4()]
    plan = batch.build_plan(jobs)
    dp = batch.DevicePlan(plan)
    dp = batch.DevicePlan(plan)             # second build: tables timed warm
    run = batch.Runner(dp)
    for _ in range(max(1, args.warmup)):
        run.batched()
    torch.cuda.synchronize()
    tb = []
    for _ in range(max(3, args.steps // 2)):
        t0 = time.perf_counter()
        res_b = run.batched()
        tb.append(time.perf_counter() - t0)
    st = run.stats_dict()
    # device time of the batched launch alone (counter fills and one
    # persistent launch per (W, delta) group), by events on the stream
    dev_ms = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run.batched(sync=False)
        e1.record()
        torch.cuda.synchronize()
        dev_ms.append(e0.elapsed_time(e1))
    dev_med = sorted(dev_ms)[len(dev_ms) // 2]
    groups = sorted({(pj.W, pj.delta) for pj in plan.jobs})
    roof = None
    if len(groups) == 1:
        # the headline kernel's ops model, with this plan's width and degree
        W, d = groups[0]
        ops = ops_model(types.SimpleNamespace(W=W, delta=d), st["pieces"], st["candidates"],
                        st["partial_quotients"], st["full_evaluations"])
        roof = {"bound": "alu", "kernel": f"k_items<{W // 32},{d},true>",
                "device_ms": dev_med, "achieved": ops / (dev_med / 1000) / 1e12,
                "peak": PEAK_INT32_OPS / 1e12, "unit": "Tops/s (int32 VALU, algorithmic)",
                "frac": ops / (dev_med / 1000) / PEAK_INT32_OPS}
    graph = run.capture()
    graph.replay()
    graph.results()
    tg = []
    for _ in range(max(3, args.steps // 2)):
        t0 = time.perf_counter()
        graph.replay()
        res_g = graph.results()
        tg.append(time.perf_counter() - t0)
    same_graph = np.array_equal(np.sort(res_g, order=["job", "sub", "piece", "k"]),
                                np.sort(res_b, order=["job", "sub", "piece", "k"]))
    run.plain()
    tp = []
    for _ in range(2):
        t0 = time.perf_counter()
        res_p = run.plain()
        tp.append(time.perf_counter() - t0)
    same = np.array_equal(np.sort(res_b, order=["job", "sub", "piece", "k"]),
                          np.sort(res_p, order=["job", "sub", "piece", "k"]))
    hr = batch.finish(plan, res_b)
    n_args = batch.args_of(plan)
    b_s, p_s = min(tb), min(tp)
    return {"workload": "16 jobs exp/log/2^x/sin, 2^30..2^38 args each, N~U[2^12,2^20] "
                        "per 2^28-arg sub-interval, eps 2^-28 RN",
            "args": n_args, "sub_intervals": sum(len(pj.subs) for pj in plan.jobs),
            "items": int(len(plan.items)), "widths": sorted({pj.W for pj in plan.jobs}),
            "degrees": sorted({pj.delta for pj in plan.jobs}),
            "batched_ms": b_s * 1000, "plain_ms": p_s * 1000,
            "batched_args_per_s": n_args / b_s, "plain_args_per_s": n_args / p_s,
            "speedup": p_s / b_s, "identical_results": bool(same),
            "graph_ms": min(tg) * 1000, "graph_speedup": p_s / min(tg),
            "graph_identical": bool(same_graph),
            "hr_cases": sum(len(v) for v in hr.values()), "candidates": st["candidates"],
            "nmdm_wave64": st["nmdm"], "roofline": roof,
            "host_prep_s": plan.prep_s, "device_tables_ms": dp.tables_ms,
            "upper_degrees": sorted({r[2] for tp, _ in plan.tables for r in tp.ranges})}


def bench_serve(args, pool):
    """2000 jobs (five functions, 2^24..2^36 arguments, eps 2^-20 or 2^-28):
    capacity with every job present at t = 0, then Poisson arrivals at 0.8 x
    that capacity; p50 / p99 latency from arrival to result."""
    import numpy as np

    import synth
    from paper_1211_3056_amd import serve
    from paper_1211_3056_amd.plan import BatchJob

    jobs = [BatchJob(**d) for d in synth.config5(n_jobs=args.serve_jobs)]
    be = serve.GpuBackend()
    srv = serve.Server(be, pool)
    t0 = time.perf_counter()
    sat = srv.serve(jobs, np.zeros(len(jobs)), realtime=False)
    cap_s = time.perf_counter() - t0
    capacity = sum(s.status == "done" for s in sat) / cap_s
    rate = 0.8 * capacity
    arrivals = synth.poisson_arrivals(len(jobs), rate)
    srv = serve.Server(be, pool)
    steps0 = be.steps
    t0 = time.perf_counter()
    states = srv.serve(jobs, arrivals)
    span = time.perf_counter() - t0
    summ = serve.summarize(states, span)
    summ.update({"workload": f"{len(jobs)} jobs, exp/log/2^x/sin/cos, 2^24..2^36 args "
                             "(log-uniform), eps 2^-20 or 2^-28 RN, Poisson arrivals",
                 "capacity_jobs_per_s": capacity, "arrival_rate_jobs_per_s": rate,
                 "device_steps": be.steps - steps0, "prep_workers": args.prep_workers,
                 "hbm_budget_bytes": srv.budget, "peak_hbm_bytes": srv.peak_used,
                 "blocked_admissions": srv.blocked_admissions,
                 "same_hr_as_saturated_run": all(np.array_equal(a.hr, b.hr)
                                                 for a, b in zip(sat, states))})
    return summ


if __name__ == "__main__":
    main()
