"""Serving loop logic on the CPU with a stand-in device backend: admission
by footprint, slots, FIFO order, failure isolation, latency bookkeeping."""
import numpy as np
import pytest

from paper_1211_3056_amd import serve
from paper_1211_3056_amd.plan import RESULT_DTYPE, BatchJob


class FakeBackend:
    """Runs nothing; records which jobs each step carried."""

    def __init__(self, free=1 << 30, fail_on=None, delay=0.0):
        self.free = free
        self.delay = delay
        self.steps = []
        self.fail_on = fail_on
        self.resident = set()
        self.max_resident = 0

    def free_memory(self):
        return self.free

    def admit(self, st):
        self.resident.add(st.job.job_id)
        self.max_resident = max(self.max_resident, len(self.resident))

    def release(self, st):
        self.resident.discard(st.job.job_id)

    def step(self, states):
        import time
        time.sleep(self.delay)
        ids = [s.job.job_id for s in states]
        self.steps.append(ids)
        if self.fail_on is not None and self.fail_on in ids:
            raise RuntimeError("device step failed")
        return [np.zeros(0, RESULT_DTYPE) for _ in states]


@pytest.fixture(scope="module")
def pool():
    p = serve.make_pool(2)
    yield p
    p.shutdown()


def _jobs(n, size=1 << 16):
    return [BatchJob("exp", 1.0 + 0.001 * i, size, 20, "rn", N=1 << 10, job_id=i) for i in range(n)]


def test_all_jobs_complete_in_arrival_order(pool):
    be = FakeBackend()
    jobs = _jobs(8)
    arrivals = np.linspace(0, 0.05, 8)
    states = serve.Server(be, pool, hbm_budget=1 << 30).serve(jobs, arrivals)
    assert [s.status for s in states] == ["done"] * 8
    assert all(s.latency >= 0 and s.t_admit >= s.arrival for s in states)
    seen = [i for step in be.steps for i in step]
    assert sorted(seen) == list(range(8))


def test_small_budget_blocks_admission(pool):
    be = FakeBackend(delay=0.05)      # device steps outlast preparations
    jobs = _jobs(6)
    fp = serve.prepare_job(jobs[0]).footprint
    srv = serve.Server(be, pool, hbm_budget=int(fp * 1.5))
    states = srv.serve(jobs, np.zeros(6), realtime=False)
    assert all(s.status == "done" for s in states)
    assert be.max_resident == 1          # only one job fits at a time
    assert srv.peak_used <= srv.budget
    assert srv.blocked_admissions > 0
    assert len(be.steps) == 6


def test_slot_cap(pool):
    be = FakeBackend()
    srv = serve.Server(be, pool, hbm_budget=1 << 30, max_resident=2)
    states = srv.serve(_jobs(5), np.zeros(5), realtime=False)
    assert all(s.status == "done" for s in states)
    assert max(len(s) for s in be.steps) <= 2


def test_failures_are_isolated(pool):
    be = FakeBackend()
    jobs = _jobs(4)
    # exp crosses 4 near ln 4: preparation refuses this range
    jobs.append(BatchJob("exp", 1.3862943, 1 << 40, 20, "rn", N=1 << 10, job_id=4))
    # larger than the budget
    jobs.append(BatchJob("exp", 1.1, 1 << 33, 20, "rn", N=1 << 10, job_id=5))
    fp = serve.prepare_job(jobs[0]).footprint
    srv = serve.Server(be, pool, hbm_budget=fp * 3)
    states = srv.serve(jobs, np.zeros(len(jobs)), realtime=False)
    st = {s.job.job_id: s for s in states}
    assert st[4].status == "failed" and "binade" in st[4].error
    assert st[5].status == "failed" and "budget" in st[5].error
    assert all(st[i].status == "done" for i in range(4))


def test_device_failure_fails_only_that_step(pool):
    be = FakeBackend(fail_on=2)
    srv = serve.Server(be, pool, hbm_budget=1 << 30, max_resident=1)
    states = srv.serve(_jobs(4), np.zeros(4), realtime=False)
    assert [s.status for s in states] == ["done", "done", "failed", "done"]


def test_summary_fields(pool):
    be = FakeBackend()
    states = serve.Server(be, pool, hbm_budget=1 << 30).serve(_jobs(3), np.zeros(3))
    s = serve.summarize(states)
    assert s["done"] == 3 and s["jobs_per_s"] > 0 and s["p99_latency_ms"] >= s["p50_latency_ms"]


def test_prepared_jobs_skip_the_pool(pool):
    be = FakeBackend()
    jobs = _jobs(5)
    preps = {j.job_id: serve.prepare_job(j) for j in jobs}
    fp = max(p.footprint for p in preps.values())
    srv = serve.Server(be, pool, hbm_budget=int(fp * 1.5))
    states = srv.serve(jobs, np.zeros(5), realtime=False, prepared=preps)
    assert all(s.status == "done" for s in states)
    assert srv.blocked_admissions >= 4 and be.max_resident == 1


def test_split_by_job_equals_filter():
    from paper_1211_3056_amd.plan import RESULT_DTYPE, canonical, split_by_job
    rng = np.random.default_rng(3)
    r = np.zeros(5000, dtype=RESULT_DTYPE)
    for f, hi in (("job", 7), ("sub", 4), ("piece", 50), ("k", 1000), ("cls", 3)):
        r[f] = rng.integers(0, hi, r.size)
    for ids in ([3, 0, 9, 6], [1 << 30, 2, 5]):
        if ids[0] == 1 << 30:
            r["job"][:100] = 1 << 30
        for jid, got in zip(ids, split_by_job(r, ids)):
            want = r[r["job"] == jid]
            assert got.tobytes() == want.tobytes()          # device order kept
            assert canonical(got).tobytes() == canonical(want).tobytes()


def test_arena_first_fit_and_merging():
    a = serve.Arena(100)
    x = a.alloc(30)
    y = a.alloc(30)
    z = a.alloc(30)
    assert (x, y, z) == (0, 30, 60) and a.alloc(11) is None and a.alloc(10) == 90
    a.release(y, 30)
    assert a.alloc(31) is None
    a.release(x, 30)                      # merges with y's range
    assert a.free == [(0, 60)]
    assert a.alloc(45) == 0
    a.release(0, 45)
    a.release(z, 30)
    a.release(90, 10)
    assert a.free == [(0, 100)] and a.free_words == 100


def test_arena_against_occupancy_map():
    """Random alloc/release sequences: ranges never overlap, every word is
    either free or held, and freed space always merges back."""
    rng = np.random.default_rng(7)
    a = serve.Arena(1000)
    held = {}
    occ = np.zeros(1000, bool)
    for _ in range(3000):
        if held and rng.random() < 0.45:
            off = list(held)[int(rng.integers(len(held)))]
            n = held.pop(off)
            assert occ[off:off + n].all()
            occ[off:off + n] = False
            a.release(off, n)
        else:
            n = int(rng.integers(1, 120))
            off = a.alloc(n)
            if off is None:
                runs = np.diff(np.flatnonzero(np.diff(np.concatenate([[1], occ.astype(int), [1]]))))
                assert n > max(runs[::2], default=0)   # no free run was long enough
                continue
            assert not occ[off:off + n].any()
            occ[off:off + n] = True
            held[off] = n
        assert a.free_words == int((~occ).sum())
        assert all(o1 + n1 < o2 for (o1, n1), (o2, _) in zip(a.free, a.free[1:]))
    for off, n in held.items():
        a.release(off, n)
    assert a.free == [(0, 1000)]


def test_prepared_job_is_deterministic_and_sized():
    job = BatchJob("sin", 1.25, 5 * (1 << 16) + 123, 12, "rn", sub_len=1 << 16,
                   N=[1000, 777, 4096, 333, 5000, 64], job_id=3)
    a, b = serve.prepare_job(job), serve.prepare_job(job)
    assert a.items.tobytes() == b.items.tobytes()
    assert [r[4].tobytes() for r in a.ranges] == [r[4].tobytes() for r in b.ranges]
    assert a.table_words == 6 * a.entries * (a.W // 64)
    assert a.footprint >= a.table_words * 8 + a.items.nbytes
    # item table offsets address the job's own table region, sub-interval by sub-interval
    assert set(a.items["table"].tolist()) == {t * a.entries * (a.W // 64) for t in range(6)}
