"""Benchmark: binary64 arguments checked per second on the 2^40-argument exp
slice (exp on [1, 1 + 2^-12), round-to-nearest, eps = 2^-32 ulp; 4096
sub-intervals of 2^28 arguments, degree-4 Taylor tables at 256 bits, degree-1
pieces of N = 2^18).

One step is one pass of the whole hot path over the slice with the initial
tables already resident in HBM: tabulation of the 2^22 pieces, degree-1
search of every piece, exact recheck of every candidate, and the result list
copied back to the host.  The fused form (one launch) is the timed step; the
plain launch chain (tabulate -> search -> recheck) is timed beside it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "binary64 args checked/sec (exp, 2^40 slice); batched vs plain speedup, p99"
PEAK_INT32_OPS = 256 * 64 * 2.4e9     # 256 CUs x 64 lanes x 2.4 GHz, one op/lane/clock
PEAK_HBM = 8.0e12                     # bytes/s

# HBM bytes per launch measured by rocprofv3 (FETCH_SIZE x 1.997 and
# WRITE_SIZE x 0.999, the factors a 1 GiB copy gives; summary under
# profiles/), valid only for the kernel sources they were taken on.
PROFILED_SOURCES = "b9d6936039a468f9"      # sha256 prefix of hr_lib.hip + hr_core.h
PROFILED_TRAFFIC = {"k_pipeline<8,4>": 4.99e6, "k_tabulate<8,4>": 78.03e6}


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
    import numpy as np
    import torch

    import synth
    from paper_1211_3056_amd import _lib, api, pipeline
    from paper_1211_3056_amd.prep import JobSpec, prepare

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe:
        probe()
        return
    spec = JobSpec(**synth.CONFIG3)
    t0 = time.time()
    P = prepare(spec, pool=pool)
    prep_s = time.time() - t0
    table, win, thr = pipeline.upload(P)
    ctx = api.context()
    dev = table.device
    stream = torch.cuda.current_stream()
    cap = 1 << 16
    RB = _lib.RESULT_BYTES
    out = torch.empty(cap * RB, dtype=torch.uint8, device=dev)
    counters = torch.zeros(9, dtype=torch.uint64, device=dev)    # count, then stats[8]
    count, stats = counters[:1], counters[1:]
    count_h = torch.zeros(1, dtype=torch.uint64).pin_memory()
    res_h = torch.zeros(cap * RB, dtype=torch.uint8).pin_memory()
    n_sub = spec.n_sub
    # Rows fetched per step: every step searches the same batch, so the last
    # count (rounded up) bounds this one; rows beyond it are fetched after
    # the loop, inside the timed region, so no result is ever left behind.
    fetch = [cap]

    def step(ev=None):
        counters.zero_()
        if ev:
            ev[0].record(stream)
        _lib.hr_pipeline(ctx, table, n_sub, spec.delta, spec.tau, spec.W, spec.N, win, thr, out,
                         cap, count, stats, stream)
        if ev:
            ev[1].record(stream)
        count_h.copy_(count, non_blocking=True)
        res_h[: fetch[0] * RB].copy_(out[: fetch[0] * RB], non_blocking=True)

    for _ in range(args.warmup):
        step()
        torch.cuda.synchronize()
        fetch[0] = min(cap, -(-max(int(count_h.numpy()[0]), 1) // 1024) * 1024)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    n_res = int(count_h.numpy()[0])
    if fetch[0] < min(n_res, cap):      # not taken while every step repeats one batch
        res_h[fetch[0] * RB: n_res * RB].copy_(out[fetch[0] * RB: n_res * RB])
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    assert n_res <= cap
    st = stats.cpu().numpy()
    pieces, cand, quot, full = int(st[0]), int(st[1]), int(st[3]), int(st[5])
    res = res_h[: n_res * _lib.RESULT_BYTES].numpy().view(api.RESULT_DTYPE)
    hr_cases = int((res["cls"] == 1).sum())
    undecided = int((res["cls"] == 2).sum())
    ms_per_step = wall * 1000 / args.steps
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
                   "form": "fused", "sub_intervals": n_sub, "pieces": pieces},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "Tops/s (int32 VALU, algorithmic)",
                     "frac": achieved / (PEAK_INT32_OPS / 1e12),
                     "traffic": profiled_traffic("k_pipeline<8,4>"),
                     "kernel": "k_pipeline<8,4>", "kernel_ms": kern_avg,
                     "kernel_ms_median": sorted(kern_ms)[len(kern_ms) // 2]},
        "hr_cases": hr_cases, "undecided": undecided, "candidates": cand,
        "full_width_evaluations": full,
        "partial_quotients": quot, "quotients_per_piece": quot / max(pieces, 1),
        "nmdm_wave64": 1.0 - quot / int(st[4]) if int(st[4]) else 0.0,
        "host_prep_s": prep_s,
        "end_to_end_args_per_s": args_total / (prep_s + ms_per_step / 1000),
    }
    line["tabulation"] = bench_tabulation(spec, table, ctx, stream, args.steps)
    if not args.no_plain:
        tp = []
        for i in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hr_plain, pst = pipeline.run_plain(P, (table, win, thr), ctx=ctx)
            torch.cuda.synchronize()
            tp.append(time.perf_counter() - t0)
        line["plain_form"] = {"ms_per_step": min(tp) * 1000,
                              "value": args_total / min(tp), "candidates": pst["candidates"],
                              "hr_cases": len(hr_plain)}
    if not args.no_batch:
        line["batch"] = bench_batch(args)
    if not args.no_serve:
        line["serving"] = bench_serve(args, pool)
    line["paper_context"] = dict(PAPER_CONTEXT)
    if not args.no_cpu_baseline:
        from oracle import hr as ohr
        from oracle import native
        from oracle.taylor import Job
        job = Job(**synth.CONFIG3)
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
    return {"kernel": kernel, "kernel_ms": ms, "pieces": pieces, "bytes": nbytes,
            "traffic": profiled_traffic(kernel), "hbm_GBps": nbytes / (ms / 1000) / 1e9,
            "hbm_frac": nbytes / (ms / 1000) / PEAK_HBM,
            "pieces_per_s": pieces / (ms / 1000)}


def probe():
    """Kernels for counter runs: a plain copy of known size (the reference
    for scaling FETCH_SIZE / WRITE_SIZE), the fused pass, the tabulation
    stage alone, the batched pass."""
    import torch

    import synth
    from paper_1211_3056_amd import api, batch, pipeline
    from paper_1211_3056_amd.prep import JobSpec, prepare

    src = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    spec = JobSpec(**synth.CONFIG3)
    P = prepare(spec)
    dev = pipeline.upload(P)
    for _ in range(3):
        pipeline.run_fused(P, dev)
    from paper_1211_3056_amd import _lib
    a_out = torch.empty(spec.n_sub * spec.tau, dtype=torch.uint64, device="cuda")
    b_out = torch.empty_like(a_out)
    for _ in range(3):
        _lib.hr_tabulate(api.context(), dev[0], spec.n_sub, spec.delta, spec.tau, spec.W,
                         a_out, b_out)
    dp = batch.DevicePlan(batch.build_plan([batch.BatchJob(**d) for d in synth.config4()]))
    run = batch.Runner(dp)
    for _ in range(3):
        run.batched()
    torch.cuda.synchronize()
    print("probe done", file=sys.stderr)


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
            "nmdm_wave64": st["nmdm"],
            "host_prep_s": plan.prep_s}


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
                 "same_hr_as_saturated_run": all(np.array_equal(a.hr, b.hr)
                                                 for a, b in zip(sat, states))})
    return summ


if __name__ == "__main__":
    main()
