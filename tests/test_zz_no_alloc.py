"""hr_search_static (no allocation; block sums in the library's fixed device
array) against hr_search on the same inputs: two calls in a row, the second
with a smaller input, each compared element by element; sizes beyond the
array are refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from paper_1211_3056_amd import _lib, api

pytestmark = pytest.mark.gpu


def _run(fn, ctx, A, B, N, lo, d, group, cap):
    dev = "cuda"
    n = len(A)
    a = api.to_dev(A, torch.uint64)
    b = api.to_dev(B, torch.uint64)
    Nd = api.to_dev(N, torch.uint32)
    lo_d = api.to_dev(lo, torch.uint64)
    d_d = api.to_dev(d, torch.uint64)
    counts = torch.full((n,), 7, dtype=torch.uint32, device=dev)
    offsets = torch.full((n,), 7, dtype=torch.uint64, device=dev)
    hits = torch.zeros(cap, dtype=torch.uint32, device=dev)
    inst = torch.zeros(cap, dtype=torch.uint32, device=dev)
    total = torch.zeros(1, dtype=torch.uint64, device=dev)
    fn(ctx, a, b, Nd, lo_d, d_d, group, counts, offsets, hits, inst, cap, total)
    torch.cuda.synchronize()
    t = int(total.cpu().numpy()[0])
    assert t <= cap
    return (counts.cpu().numpy(), offsets.cpu().numpy(), hits[:t].cpu().numpy(),
            inst[:t].cpu().numpy(), t)


def _case(seed, n, group):
    A, B, N, lo, D = synth.adversarial_instances(seed, n, max_N=1000)
    ng = -(-n // group)
    return A, B, N, lo[:ng].copy(), D[:ng].copy()


def test_static_scratch_search_equals_search_twice():
    ctx = api.context()
    for seed, n, group in ((31, 200_003, 3), (32, 40_001, 1)):   # second call smaller
        A, B, N, lo, D = _case(seed, n, group)
        cap = 1 << 26
        ref = _run(_lib.hr_search, ctx, A, B, N, lo, D, group, cap)
        got = _run(_lib.hr_search_static, ctx, A, B, N, lo, D, group, cap)
        assert ref[4] == got[4] > 0
        for x, y in zip(ref[:4], got[:4]):
            assert np.array_equal(x, y)


def test_static_scratch_config1_and_limit():
    ctx = api.context()
    A, B, N, D = synth.config1()
    n = len(A)
    ref = _run(_lib.hr_search, ctx, A, B, N, np.zeros(1, np.uint64), np.full(1, D, np.uint64),
               n, 1 << 12)
    got = _run(_lib.hr_search_static, ctx, A, B, N, np.zeros(1, np.uint64),
               np.full(1, D, np.uint64), n, 1 << 12)
    for x, y in zip(ref[:4], got[:4]):
        assert np.array_equal(x, y)
    # one instance more than the array allows: refused on the host
    big = _lib.HR_STATIC_MAX_INSTANCES + 1
    a = torch.zeros(big, dtype=torch.uint64, device="cuda")
    Nd = torch.zeros(big, dtype=torch.uint32, device="cuda")
    d = torch.zeros(1, dtype=torch.uint64, device="cuda")
    counts = torch.zeros(big, dtype=torch.uint32, device="cuda")
    offsets = torch.zeros(big, dtype=torch.uint64, device="cuda")
    hits = torch.zeros(1, dtype=torch.uint32, device="cuda")
    total = torch.zeros(1, dtype=torch.uint64, device="cuda")
    with pytest.raises(_lib.HRError) as e:
        _lib.hr_search_static(ctx, a, a, Nd, None, d, big, counts, offsets, hits, None, 1, total)
    assert e.value.status == _lib.HR_ESCRATCH
