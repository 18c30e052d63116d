"""GPU parity of hr_search against the brute-force oracle (bit-exact)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import native

pytestmark = pytest.mark.gpu


def _dev(x, dt):
    from paper_1211_3056_amd import api
    return api.to_dev(x, dt)


def _gpu(A, B, N, D, lo=None, group=None, cap=None):
    from paper_1211_3056_amd import api
    lo_t = None
    if lo is not None:
        lo_t = _dev(lo, torch.uint64)
    D_t = _dev(D, torch.uint64) if isinstance(D, np.ndarray) else D
    counts, offsets, hits, inst = api.search(_dev(A, torch.uint64), _dev(B, torch.uint64),
                                             _dev(N, torch.uint32), D_t, lo=lo_t, group=group,
                                             cap=cap, with_inst=True)
    return (counts.cpu().numpy(), offsets.cpu().numpy(), hits.cpu().numpy(), inst.cpu().numpy())


def _expand(arr, group, n):
    return np.repeat(arr, group)[:n]


def test_config1_parity():
    """4096 random instances, N = 2^16, d = 2^-20: every hit, bit for bit."""
    A, B, N, D = synth.config1()
    n = A.size
    c, o, h, inst = _gpu(A, B, N, D)
    rc, ro, rk = native.brute_hits_many(A, B, N, np.zeros(n, np.uint64), np.full(n, D, np.uint64))
    assert np.array_equal(c, rc)
    assert np.array_equal(o, ro)
    assert np.array_equal(h, rk)
    assert np.array_equal(inst, np.repeat(np.arange(n, dtype=np.uint32), rc))
    assert 150 < rk.size < 400          # about 256 expected


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_adversarial_instances(seed):
    """Degenerate a (0, powers of two, short periods, near 0 or 1), N from 0
    to thousands, windows from empty to the whole circle, per-instance lo."""
    A, B, N, lo, D = synth.adversarial_instances(seed, 3000)
    c, o, h, _ = _gpu(A, B, N, D, lo=lo, group=1)
    rc, ro, rk = native.brute_hits_many(A, B, N, lo, D)
    assert np.array_equal(c, rc)
    assert np.array_equal(o, ro)
    assert np.array_equal(h, rk)


@pytest.mark.parametrize("seed", [31, 32])
def test_wave_coherent_slopes(seed):
    """Waves whose 64 slopes nearly agree, as for adjacent pieces (whole
    waves take the walk's subtraction path while every quotient is at most
    2), and every other wave with one unrelated slope (the wave takes the
    division path at the steps that lane needs): every hit, bit for bit."""
    A, B, N, D = synth.wave_slopes(seed, 64)
    n = A.size
    c, o, h, _ = _gpu(A, B, N, D)
    rc, ro, rk = native.brute_hits_many(A, B, N, np.zeros(n, np.uint64), np.full(n, D, np.uint64))
    assert np.array_equal(c, rc)
    assert np.array_equal(o, ro)
    assert np.array_equal(h, rk)
    assert rk.size > 4 * n // 2         # about 4 hits per instance


def test_grouped_windows_and_ragged_tail():
    g = synth.rng(5)
    n, group = 1000 + 37, 7            # ragged last group and last block
    A = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    N = g.integers(1, 1 << 14, n).astype(np.uint32)
    ng = (n + group - 1) // group
    lo = g.integers(0, 2 ** 64, ng, dtype=np.uint64, endpoint=False)
    D = (g.integers(1, 1 << 20, ng).astype(np.uint64) << np.uint64(40))
    c, o, h, _ = _gpu(A, B, N, D, lo=lo, group=group)
    rc, ro, rk = native.brute_hits_many(A, B, N, _expand(lo, group, n), _expand(D, group, n))
    assert np.array_equal(c, rc) and np.array_equal(h, rk)


def test_capacity_protocol():
    """Hits beyond cap are dropped, total stays exact, the prefix is right."""
    from paper_1211_3056_amd import _lib, api
    A, B, N, D = synth.config1(seed=3, n=2048, N=1 << 14, D=1 << 52)
    ctx = api.context()
    a, b, Nt = _dev(A, torch.uint64), _dev(B, torch.uint64), _dev(N, torch.uint32)
    d = _dev(np.array([D], np.uint64), torch.uint64)
    counts = torch.empty(A.size, dtype=torch.uint32, device="cuda")
    offs = torch.empty(A.size, dtype=torch.uint64, device="cuda")
    total = torch.zeros(1, dtype=torch.uint64, device="cuda")
    cap = 100
    hits = _dev(np.full(cap + 16, 0xFFFFFFFF, np.uint32), torch.uint32)
    _lib.hr_search(ctx, a, b, Nt, None, d, A.size, counts, offs, hits, None, cap, total)
    torch.cuda.synchronize()
    rc, ro, rk = native.brute_hits_many(A, B, N, np.zeros(A.size, np.uint64), np.full(A.size, D, np.uint64))
    assert int(total.cpu().numpy()[0]) == rk.size > cap
    h = hits.cpu().numpy()
    assert np.array_equal(h[:cap], rk[:cap])
    assert np.all(h[cap:] == 0xFFFFFFFF)


def test_deterministic_bytes():
    A, B, N, D = synth.config1(seed=9, n=4096, N=1 << 15, D=1 << 50)
    r1 = _gpu(A, B, N, D)
    r2 = _gpu(A, B, N, D)
    for x, y in zip(r1, r2):
        assert x.tobytes() == y.tobytes()


def test_large_n_sampled():
    """N up to 2^28 per instance: brute force on a handful of instances."""
    g = synth.rng(21)
    n = 6
    A = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    N = np.array([1 << 28, (1 << 28) - 3, 1 << 27, 1 << 26, 12345678, 1 << 20], np.uint32)
    D = np.uint64(1 << 38)
    c, o, h, _ = _gpu(A, B, N, int(D))
    rc, ro, rk = native.brute_hits_many(A, B, N, np.zeros(n, np.uint64), np.full(n, D, np.uint64))
    assert np.array_equal(c, rc) and np.array_equal(h, rk)


def test_maximum_n_properties():
    """N = 2^32 - 1: every reported k is in the window, and the count matches
    the area N d / 2^64 within Poisson noise over many instances."""
    g = synth.rng(22)
    n = 256
    A = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    B = g.integers(0, 2 ** 64, n, dtype=np.uint64, endpoint=False)
    N = np.full(n, 2 ** 32 - 1, np.uint32)
    D = 1 << 30                          # ~0.25 hits per instance
    c, o, h, inst = _gpu(A, B, N, D)
    with np.errstate(over="ignore"):
        dist = B[inst] - h.astype(np.uint64) * A[inst]
    assert np.all(dist < np.uint64(D))
    assert np.all(h < N[inst])
    exp = n * (2 ** 32 - 1) * D / 2 ** 64
    assert abs(h.size - exp) < 6 * exp ** 0.5 + 3
    # hits of one instance are distinct and sorted by distance
    for i in range(n):
        s = slice(int(o[i]), int(o[i]) + int(c[i]))
        assert len(set(h[s].tolist())) == c[i]
        assert np.all(np.diff(dist[s].astype(np.float64)) >= 0)


def test_empty_input():
    from paper_1211_3056_amd import api
    e64 = torch.empty(0, dtype=torch.uint64, device="cuda")
    e32 = torch.empty(0, dtype=torch.uint32, device="cuda")
    c, o, h, _ = api.search(e64, e64, e32, 1 << 40)
    assert c.numel() == 0 and h.numel() == 0


def test_device_quotient_routine_exact():
    """The partial-quotient routine (binary64 reciprocal estimate + exact
    correction) against Python integer division, over every scale of
    quotient, exact multiples, off-by-one neighbours and saturation."""
    from paper_1211_3056_amd import _lib, api
    g = synth.rng(77)
    M = 1 << 64
    nums, dens = [], []
    for _ in range(200000):
        den = int(g.integers(1, 2 ** 63)) >> int(g.integers(0, 63))
        den = max(den, 1)
        kind = int(g.integers(0, 4))
        if kind == 0:
            num = int(g.integers(0, 2 ** 63)) * 2 + int(g.integers(0, 2))
        elif kind == 1:                       # exact multiple and neighbours
            k = int(g.integers(0, 1 << 34))
            num = min(k * den + int(g.integers(-1, 2)), M - 1)
        elif kind == 2:                       # quotient near the cap
            k = int(g.integers((1 << 32) - 8, (1 << 32) + 8))
            num = min(k * den - int(g.integers(0, 2)), M - 1)
        else:                                 # num near 2^64
            num = M - 1 - int(g.integers(0, 1 << 20))
        nums.append(max(num, 0) % M)
        dens.append(den)
    nums += [M - 1, M - 1, M - 2, 0, 1, (1 << 63) + 1]
    dens += [1, M - 1, M - 1, 5, 1, (1 << 63) - 1]
    num_t = api.to_dev(np.array(nums, np.uint64), torch.uint64)
    den_t = api.to_dev(np.array(dens, np.uint64), torch.uint64)
    for cap in (1, 65536, (1 << 32) - 1, 3000000000):
        out = torch.empty(len(nums), dtype=torch.uint64, device="cuda")
        rem = torch.empty(len(nums), dtype=torch.uint64, device="cuda")
        _lib.hr_quot_check(api.context(), num_t, den_t, cap, out, rem)
        got, got_r = out.cpu().numpy(), rem.cpu().numpy()
        want = np.array([min(n // d, cap) for n, d in zip(nums, dens)], np.uint64)
        want_r = np.array([n % d if n // d < cap else M - 1 for n, d in zip(nums, dens)], np.uint64)
        bad = np.nonzero((got != want) | (got_r != want_r))[0]
        assert bad.size == 0, [(nums[i], dens[i], cap, int(got[i]), int(want[i])) for i in bad[:5]]


def test_search_steps_match_pipeline_statistics():
    """hr_search_steps on the tabulated pieces of a small exp range counts
    the same partial quotients as the fused pass's statistics (both run
    the closest-point walk on identical (a, b, N, window))."""
    import numpy as np
    import torch

    from paper_1211_3056_amd import _lib, api, pipeline
    from paper_1211_3056_amd.prep import JobSpec, prepare
    spec = JobSpec("exp", 1.0, 1 << 22, 12, "rn", 1 << 10, 1 << 6, 3, 192)
    P = prepare(spec)
    table, win, thr = pipeline.upload(P)
    ctx = api.context()
    _, st = api.pipeline(table, spec.n_sub, spec.delta, spec.tau, spec.W, spec.N, win, thr)
    stats = torch.zeros(8, dtype=torch.uint64, device="cuda")
    out = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.uint64, device="cuda")
    _lib.hr_pipeline(ctx, table, spec.n_sub, spec.delta, spec.tau, spec.W, spec.N, win, thr,
                     out, (1 << 20) // _lib.RESULT_BYTES, count, stats)
    a, b = api.tabulate(table, spec.n_sub, spec.delta, spec.tau, spec.W)
    n = spec.n_sub * spec.tau
    N = api.to_dev(np.full(n, spec.N, np.uint32), torch.uint32)
    lo = api.to_dev(P.win[:, 0], torch.uint64)
    d = api.to_dev(P.win[:, 1], torch.uint64)
    steps = torch.empty(n, dtype=torch.uint32, device="cuda")
    _lib.hr_search_steps(ctx, a, b, N, lo, d, spec.tau, steps)
    torch.cuda.synchronize()
    s = steps.cpu().numpy().astype(np.int64)
    assert s.min() >= 1 and s.max() <= 64
    assert int(s.sum()) == int(stats.cpu().numpy()[3])
