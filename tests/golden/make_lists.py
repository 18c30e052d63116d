"""Write the oracle's complete HR-case lists of the full-size workloads.

Calls only ``oracle/`` (and ``synth`` for the seeded job descriptions): the
three-phase pipeline oracle of Sec. 4.1 on every sub-interval, each
sub-interval in its own worker process (one thread each), then the exact
per-argument test (Def. 2-3, Sec. 3.1) for arguments left outside the
oracle's sub-interval grid.

    python tests/golden/make_lists.py config3 [--workers 7]
    python tests/golden/make_lists.py table3  [--workers 7]
    python tests/golden/make_lists.py config4 [--workers 7]
    python tests/golden/make_lists.py table3_s31 [--workers 7]

Workloads (binary64 arguments X = X0 + m ulp(X0); the lists hold the
offsets m):
  config3  exp on [1, 1 + 2^-12) (2^40 arguments), round to nearest,
           eps = 2^-32 ulp; oracle tables of degree 4 at 256 bits,
           sub-intervals of 2^28 arguments, pieces of 2^18.
  table3   the workload of Table 3: exp on the closed interval
           [1, 1 + 2^-13] (2^39 + 1 arguments), directed breakpoints,
           eps = 2^-32 ulp; degree 3 at 192 bits, pieces of 2^15; the last
           argument (1 + 2^-13 itself) by the per-argument test.
  table3_s31  the table3 range at eps = 2^-31 ulp, each case with its
           distance to the nearest representable number (in ulps): the cases
           nearest to the 2^-32 threshold, for comparing counts with the
           paper's Table 3.
  config4  the 12 exp, 2^x and sin jobs of the batched workload (2^30 ..
           2^38 arguments each), round to nearest, eps = 2^-28 ulp; the
           oracle cuts every job into its own sub-intervals of 2^28
           arguments and pieces of 2^16, degree 3 at 128 bits.  The HR set
           of a range does not depend on how it is cut.
  config4_log  the four log jobs of the same workload (2688
           sub-intervals), the same way.  Near 3 the scaled values of log
           advance by about 2/3 ulp per argument, so they sit close to a
           three-point lattice mod 1 that defeats the oracle's Alg. 1 filter
           on many pieces; its exhaustive scan then takes up to 80 s on the
           sub-intervals next to 3 and 3-6 s elsewhere.
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _jobs(name):
    """[(job_id, oracle Job, extra offsets checked one by one)]."""
    import synth
    from oracle.taylor import Job
    if name == "config3":
        return [(0, Job(**synth.CONFIG3), [])]
    if name == "table3":
        n = 1 << 39
        return [(0, Job("exp", 1.0, n, 32, "dir", 1 << 15, 1 << 13, 3, 192), [n])]
    if name == "table3_s31":
        n = 1 << 39
        return [(0, Job("exp", 1.0, n, 31, "dir", 1 << 15, 1 << 13, 3, 192), [n])]
    if name in ("config4", "config4_log"):
        out = []
        for d in synth.config4():
            if (d["fname"] == "log") != (name == "config4_log"):
                continue
            out.append((d["job_id"], Job(d["fname"], d["X0"], d["count"], d["s"], d["mode"],
                                         1 << 16, 1 << 12, 3, 128), []))
        return out
    raise ValueError(name)


def _run_sub(task):
    from oracle import hr as ohr
    job_id, job, t = task
    return job_id, t, ohr.pipeline(job, subs=[t], threads=1)


def _run_single(task):
    from oracle import hr as ohr
    job_id, job, m = task
    return job_id, m, ohr.decide(job, m)


def generate(name, workers):
    jobs = _jobs(name)
    tasks = [(jid, job, t) for jid, job, _ in jobs for t in range(job.n_sub)]
    # jobs in order, each job's sub-intervals in order (for the log jobs the
    # slowest ones, next to 3, come first)
    found = {jid: [] for jid, _, _ in jobs}
    t0 = time.time()
    done = 0
    with ProcessPoolExecutor(workers) as ex:
        for jid, t, hr in ex.map(_run_sub, tasks, chunksize=4):
            found[jid] += hr
            done += 1
            if done % 256 == 0 or done == len(tasks):
                print(f"{name}: {done}/{len(tasks)} sub-intervals, "
                      f"{sum(map(len, found.values()))} cases, {time.time() - t0:.0f} s",
                      flush=True)
        singles = [(jid, job, m) for jid, job, extra in jobs for m in extra]
        for jid, m, hit in ex.map(_run_single, singles):
            if hit:
                found[jid].append(m)
    return jobs, found, time.time() - t0


def _distance_col(job, m):
    """' <distance in ulps, 17 significant digits>' for the lists that keep it."""
    import mpmath

    from oracle import hr as ohr
    with mpmath.workprec(192):
        return " " + mpmath.nstr(ohr.distance(job, m), 17)


def write(name, jobs, found, secs):
    path = os.path.join(HERE, f"hr_{name}.txt")
    with_dist = name.endswith("_s31")
    with open(path, "w") as f:
        f.write(f"# Oracle HR-case list of the '{name}' workload (module docstring of\n"
                f"# tests/golden/make_lists.py), written by\n"
                f"#   python tests/golden/make_lists.py {name}\n"
                f"# which calls only oracle/ (three-phase pipeline, Sec. 4.1; exact\n"
                f"# per-argument decisions, Def. 2-3).  {secs:.0f} s of oracle time.\n")
        f.write("# columns: job fname X0 count s mode | offset m (X = X0 + m ulp(X0))"
                + (" distance/ulp" if with_dist else "") + "\n")
        for jid, job, extra in jobs:
            count = job.count + len(extra)
            for m in sorted(found[jid]):
                dist = _distance_col(job, m) if with_dist else ""
                f.write(f"{jid} {job.fname} {job.X0!r} {count} {job.s} {job.mode} | {m}{dist}\n")
            if not found[jid]:
                f.write(f"{jid} {job.fname} {job.X0!r} {count} {job.s} {job.mode} | -\n")
    return path


def main():
    p = argparse.ArgumentParser()
    p.add_argument("name", choices=("config3", "table3", "config4", "config4_log", "table3_s31"))
    p.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    a = p.parse_args()
    jobs, found, secs = generate(a.name, a.workers)
    print(write(a.name, jobs, found, secs))


if __name__ == "__main__":
    main()
