"""GPU parity of hr_tabulate and hr_recheck against the oracle (bit-exact)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import tabulate as otab
from oracle.taylor import Job, initial_table

pytestmark = pytest.mark.gpu


def _words(tables_np, delta):
    """uint64 (n_sub, E, L) -> per sub-interval T[j][l] as Python ints."""
    n_sub, E, L = tables_np.shape
    out = []
    for s in range(n_sub):
        flat = [sum(int(tables_np[s, e, l]) << (64 * l) for l in range(L)) for e in range(E)]
        T, pos = [], 0
        for j in range(delta + 1):
            T.append(flat[pos:pos + delta - j + 1])
            pos += delta - j + 1
        out.append(T)
    return out


def _pack(T, W):
    L = W // 64
    flat = [v for row in T for v in row]
    return np.array([[(v >> (64 * l)) & ((1 << 64) - 1) for l in range(L)] for v in flat], np.uint64)


@pytest.mark.parametrize("W", [128, 192, 256])
@pytest.mark.parametrize("delta,tau", [(1, 5), (2, 77), (3, 256), (4, 1000), (5, 130), (6, 33)])
def test_tabulate_random_tables(W, delta, tau):
    from paper_1211_3056_amd import api
    n_sub = 3
    tabs = synth.random_tables(100 * W + delta, n_sub, delta, W)
    a, b = api.tabulate(api.to_dev(tabs.reshape(-1), torch.uint64), n_sub, delta, tau, W)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    ra, rb = otab.tabulate(_words(tabs, delta), delta, tau, W)
    assert a.tolist() == ra and b.tolist() == rb


@pytest.mark.parametrize("W,delta,tau", [(256, 4, 66000), (192, 5, 4500), (128, 6, 1500),
                                         (256, 6, 700)])
def test_tabulate_start_paths(W, delta, tau):
    """Both packet starts: lanes whose first piece i0 has i0 + 32 delta below
    the 64-bit binomial limit of delta (2^16, 2^12, 2^10) take the composed
    shift and step change with 64-bit multipliers, later ones the 128-bit
    shift and a second pass; a sub-interval of tau pieces crosses the limit
    (tau = 700 at degree 6 stays just below it)."""
    from paper_1211_3056_amd import api
    n_sub = 2
    tabs = synth.random_tables(7 * W + delta, n_sub, delta, W)
    a, b = api.tabulate(api.to_dev(tabs.reshape(-1), torch.uint64), n_sub, delta, tau, W)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    ra, rb = otab.tabulate(_words(tabs, delta), delta, tau, W)
    assert a.tolist() == ra and b.tolist() == rb


def test_tabulate_exp_tables_from_oracle():
    """Tables of exp written by the oracle (degree 4, 256 bits, tau = 1024)."""
    from paper_1211_3056_amd import api
    job = Job("exp", 1.0, 1 << 40, 32, "rn", 1 << 18, 1 << 10, 4, 256)
    subs = [0, 2047, 4095]
    Ts = [initial_table(job, t) for t in subs]
    tabs = np.stack([_pack(T, 256) for T in Ts])
    a, b = api.tabulate(api.to_dev(tabs.reshape(-1), torch.uint64), len(subs), 4, 1 << 10, 256)
    ra, rb = otab.tabulate(Ts, 4, 1 << 10, 256)
    assert a.cpu().numpy().tolist() == ra and b.cpu().numpy().tolist() == rb


@pytest.mark.parametrize("W,delta", [(128, 3), (192, 3), (256, 4), (256, 6)])
def test_recheck_random(W, delta):
    from paper_1211_3056_amd import api
    n_sub, tau, N = 4, 300, 1 << 14
    tabs = synth.random_tables(7 * W + delta, n_sub, delta, W)
    g = synth.rng(W + delta)
    nc = 3000
    inst = g.integers(0, n_sub * tau, nc).astype(np.uint32)
    k = g.integers(0, N, nc).astype(np.uint32)
    k[:5] = [0, 1, N - 1, 2, 3]
    thr = np.zeros((n_sub, 4), np.uint64)
    thr[:, 0], thr[:, 1] = 1 << 40, 1 << 62
    thr[:, 2], thr[:, 3] = (1 << 62) + (1 << 40), (1 << 64) - (1 << 40)
    value, cls = api.recheck(api.to_dev(tabs.reshape(-1), torch.uint64), n_sub, delta, tau, W,
                             api.to_dev(inst, torch.uint32), api.to_dev(k, torch.uint32), N - 1,
                             api.to_dev(thr.reshape(-1), torch.uint64))
    value, cls = value.cpu().numpy(), cls.cpu().numpy()
    Ts = _words(tabs, delta)
    for c in range(nc):
        s, i = divmod(int(inst[c]), tau)
        V = otab.evaluate(otab.straightforward_rows(Ts[s], delta, i, W), int(k[c]), W)
        t = otab.top64(V, W)
        assert int(value[c]) == t
        want = 1 if thr[s, 0] <= t <= thr[s, 1] else (0 if thr[s, 2] <= t <= thr[s, 3] else 2)
        assert int(cls[c]) == want


def test_tabulate_config3_full_size_sampled():
    """All 2^22 pieces of the 2^40-argument exp workload on the device from
    the product's tables; sampled pieces against the oracle's own tables."""
    from paper_1211_3056_amd import api
    from paper_1211_3056_amd.prep import JobSpec, prepare
    spec = JobSpec(**synth.CONFIG3)
    P = prepare(spec)
    a, b = api.tabulate(api.to_dev(P.tables.reshape(-1), torch.uint64), spec.n_sub, spec.delta,
                        spec.tau, spec.W)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    job = Job(**synth.CONFIG3)
    g = synth.rng(33)
    for t in [0, 1, 4095] + g.integers(0, spec.n_sub, 5).tolist():
        T = initial_table(job, int(t))
        for i in [0, 1, 511, 1023] + g.integers(0, spec.tau, 4).tolist():
            ra, rb = otab.piece_ab(otab.straightforward_rows(T, 4, int(i), 256), 256)
            assert (int(a[t * spec.tau + i]), int(b[t * spec.tau + i])) == (ra, rb)


@pytest.mark.parametrize("W,delta,n_sub,tau", [(256, 4, 4200, 1001), (192, 3, 4200, 1000),
                                               (128, 2, 262144, 9)])
def test_tabulate_long_packets_ragged(W, delta, n_sub, tau):
    """Inputs large enough for 16 pieces per lane, staged in two parts of 8,
    with sub-intervals that end inside a packet (tau = 1001: a last packet of
    9, the second part holding one piece; tau = 1000: a last packet of 8, no
    second part; tau = 9: every packet split 8 + 1).  Every output is written
    (none keeps the fill value) and sampled pieces equal the oracle's."""
    from paper_1211_3056_amd import _lib, api
    # the library takes 16 pieces per lane once that still leaves 2^18 lanes
    assert n_sub * -(-tau // 16) >= 1 << 18
    tabs = synth.random_tables(77 * W + tau, n_sub, delta, W)
    fill = 0x5A5A5A5A5A5A5A5A                    # below 2^63: the same bits as int64
    a = torch.full((n_sub * tau,), fill, dtype=torch.int64, device="cuda").view(torch.uint64)
    b = torch.full((n_sub * tau,), fill, dtype=torch.int64, device="cuda").view(torch.uint64)
    _lib.hr_tabulate(api.context(), api.to_dev(tabs.reshape(-1), torch.uint64), n_sub, delta, tau,
                     W, a, b)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert not np.any(a == np.uint64(fill)) and not np.any(b == np.uint64(fill))
    g = synth.rng(tau + W)
    subs = sorted({0, 1, 63, 64, n_sub - 2, n_sub - 1} | set(g.integers(0, n_sub, 6).tolist()))
    edge = [0, 1, 7, 8, 9, 15, 16, 17, tau - 9, tau - 8, tau - 2, tau - 1]
    for t in subs:
        T = _words(tabs[t:t + 1], delta)[0]
        for i in sorted({i for i in edge if 0 <= i < tau} | set(g.integers(0, tau, 4).tolist())):
            ra, rb = otab.piece_ab(otab.straightforward_rows(T, delta, int(i), W), W)
            assert (int(a[t * tau + i]), int(b[t * tau + i])) == (ra, rb), (t, i)


@pytest.mark.parametrize("W,delta,N", [(256, 4, 1 << 12), (192, 3, 1 << 14), (256, 6, 1 << 10),
                                       (128, 3, 1 << 14)])
def test_fused_classes_at_threshold_boundaries(W, delta, N):
    """Thresholds placed on exact candidate values and up to 8 units either
    side: the fused pass (rejection from the top 128 bits with its error
    bound, else full width) must classify every candidate exactly as the
    plain full-width recheck does, including an HR band that overlaps the
    reject band."""
    from paper_1211_3056_amd import api
    n_sub, tau = 3, 64
    tabs = synth.random_tables(31 * W + delta, n_sub, delta, W)
    table = api.to_dev(tabs.reshape(-1), torch.uint64)
    g = synth.rng(W * 7 + delta)
    win = np.zeros((n_sub, 2), np.uint64)
    win[:, 0] = g.integers(0, 2 ** 64, n_sub, dtype=np.uint64, endpoint=False)
    win[:, 1] = np.uint64((1 << 64) // N * 16)               # ~16 candidates a piece
    a, b = api.tabulate(table, n_sub, delta, tau, W)
    Nt = torch.full((n_sub * tau,), N, dtype=torch.uint32, device="cuda")
    _, _, hits, inst = api.search(a, b, Nt, api.to_dev(win[:, 1], torch.uint64),
                                  lo=api.to_dev(win[:, 0], torch.uint64), group=tau,
                                  with_inst=True)
    dummy = api.to_dev(np.zeros(4 * n_sub, np.uint64), torch.uint64)
    value, _ = api.recheck(table, n_sub, delta, tau, W, inst, hits, N - 1, dummy)
    value, inst_h, k_h = value.cpu().numpy(), inst.cpu().numpy(), hits.cpu().numpy()
    sub_h = inst_h // tau
    assert value.size > 2000
    for overlap in (False, True):
        for off in range(-8, 9):
            thr = np.zeros((n_sub, 4), np.uint64)
            for s in range(n_sub):
                v = np.sort(value[sub_h == s])
                q = lambda f: int(v[int(f * (v.size - 1))])
                shift = lambda x, o: np.uint64(min(max(x + o, 0), (1 << 64) - 1))
                thr[s, 2], thr[s, 3] = shift(q(0.2), off), shift(q(0.7), -off)
                if overlap:
                    thr[s, 0], thr[s, 1] = shift(q(0.6), -off), shift(q(0.8), off)
                else:
                    thr[s, 0], thr[s, 1] = shift(q(0.75), off), shift(q(0.9), -off)
            thr_t = api.to_dev(thr.reshape(-1), torch.uint64)
            _, want_cls = api.recheck(table, n_sub, delta, tau, W, inst, hits, N - 1, thr_t)
            want_cls = want_cls.cpu().numpy()
            keep = want_cls != 0
            want = sorted(zip(sub_h[keep].tolist(), (inst_h[keep] % tau).tolist(),
                              k_h[keep].tolist(), want_cls[keep].tolist(), value[keep].tolist()))
            res, _ = api.pipeline(table, n_sub, delta, tau, W, N,
                                  api.to_dev(win.reshape(-1), torch.uint64), thr_t)
            got = sorted(zip(res["sub"].tolist(), res["piece"].tolist(), res["k"].tolist(),
                             res["cls"].tolist(), res["value"].tolist()))
            assert got == want, (overlap, off)
