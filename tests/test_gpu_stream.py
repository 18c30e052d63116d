"""Streamed batched launches (hr_batch_open / submit / poll / wait / close):
launches queued while others run give, together, the records of one
batched launch over the same items; a launch submitted while another is in
flight gives the same bytes as alone; tickets complete in order."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from paper_1211_3056_amd.plan import canonical

pytestmark = pytest.mark.gpu


def _plan():
    from paper_1211_3056_amd import batch
    jobs = [batch.BatchJob(**d) for d in synth.config4(scale_log2=14, N_scale_log2=6, s=14)]
    return batch.DevicePlan(batch.build_plan(jobs, target_items=1024))


def _records(out, count):
    from paper_1211_3056_amd import _lib, api
    n = api._u64_scalar(count)
    return out[: n * _lib.RESULT_BYTES].cpu().numpy().view(api.RESULT_DTYPE).copy()


def test_streamed_launches_equal_one_batched_launch():
    from paper_1211_3056_amd import _lib, api, batch
    dp = _plan()
    W, d, first, n = max(dp.groups, key=lambda g: g[3])      # the largest (W, delta) group
    ref_all = canonical(batch.Runner(dp).batched())
    # the group's own records: its items alone in one batched launch
    IB = _lib.ITEM_BYTES
    out = torch.empty((1 << 18) * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.uint64, device="cuda")
    _lib.hr_batch_run(api.context(), dp.pool, dp.sorted_items[first * IB:(first + n) * IB], n, W, d,
                      _lib.HR_WAVES_FILL, out, 1 << 18, count, None)
    ref = canonical(_records(out, count))
    assert 0 < len(ref) <= len(ref_all)
    bs = _lib.BatchStream(api.context(), slots=3)
    cuts = [0, n // 5, n // 2, n]
    bufs, tickets = [], []
    for lo, hi in zip(cuts, cuts[1:]):
        items = dp.sorted_items[(first + lo) * IB:(first + hi) * IB]
        out = torch.empty((1 << 18) * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda")
        count = torch.zeros(1, dtype=torch.uint64, device="cuda")
        t = bs.submit(dp.pool, items, hi - lo, W, d, out, 1 << 18, count,
                      after_stream=torch.cuda.current_stream())
        assert t is not None
        tickets.append(t)
        bufs.append((out, count))
    assert tickets == [1, 2, 3]
    bs.wait(3)
    assert bs.poll() == 3
    got = canonical(np.concatenate([_records(o, c) for o, c in bufs]))
    assert got.tobytes() == ref.tobytes()
    bs.close()


def test_launch_submitted_in_flight_equals_alone():
    """A job's items submitted while a large launch runs give the same bytes
    as the same items launched alone; with one slot, the second submit waits
    for the first (None until it is over)."""
    from paper_1211_3056_amd import _lib, api
    dp = _plan()
    W, d, first, n = max(dp.groups, key=lambda g: g[3])
    IB = _lib.ITEM_BYTES
    small = dp.sorted_items[(first + n - 50) * IB:(first + n) * IB]
    big = dp.sorted_items[first * IB:(first + n - 50) * IB]

    def buf():
        return (torch.empty((1 << 18) * _lib.RESULT_BYTES, dtype=torch.uint8, device="cuda"),
                torch.zeros(1, dtype=torch.uint64, device="cuda"))
    bs = _lib.BatchStream(api.context(), slots=4)
    o1, c1 = buf()
    o2, c2 = buf()
    t1 = bs.submit(dp.pool, big, n - 50, W, d, o1, 1 << 18, c1)
    t2 = bs.submit(dp.pool, small, 50, W, d, o2, 1 << 18, c2)
    bs.wait(t2)
    bs.wait(t1)
    in_flight = canonical(_records(o2, c2))
    o3, c3 = buf()
    t3 = bs.submit(dp.pool, small, 50, W, d, o3, 1 << 18, c3)
    bs.wait(t3)
    assert canonical(_records(o3, c3)).tobytes() == in_flight.tobytes()
    bs.close()
    one = _lib.BatchStream(api.context(), slots=1)
    ta = one.submit(dp.pool, big, n - 50, W, d, o1, 1 << 18, c1)
    tb = one.submit(dp.pool, small, 50, W, d, o2, 1 << 18, c2)
    if tb is None:                   # the slot is still busy
        one.wait(ta)
        tb = one.submit(dp.pool, small, 50, W, d, o2, 1 << 18, c2)
    one.wait(tb)
    assert one.poll() == tb == 2
    assert canonical(_records(o2, c2)).tobytes() == in_flight.tobytes()
    one.close()
