"""The paper's lower-bound tests on the device (hr_filter: Lefevre's with
swap, Alg. 1/3; the regular one unrolled, Alg. 4) against the oracle's Alg. 1
and Alg. 4 instance by instance: certification, distance value at exit and
main-loop passes, on degenerate instances and on tabulated pieces of an exp
range; a certified instance never has a hit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle.search import lefevre_alg1, regular_alg4

pytestmark = pytest.mark.gpu


def _device(alg, A, B, N, lo, D, group):
    from paper_1211_3056_amd import _lib, api
    n = len(A)
    passed = torch.empty(n, dtype=torch.uint8, device="cuda")
    d_out = torch.empty(n, dtype=torch.uint64, device="cuda")
    iters = torch.empty(n, dtype=torch.uint32, device="cuda")
    _lib.hr_filter(api.context(), alg, api.to_dev(A, torch.uint64), api.to_dev(B, torch.uint64),
                   api.to_dev(N, torch.uint32), api.to_dev(lo, torch.uint64),
                   api.to_dev(D, torch.uint64), group, passed, d_out, iters)
    torch.cuda.synchronize()
    return passed.cpu().numpy(), d_out.cpu().numpy(), iters.cpu().numpy()


@pytest.mark.parametrize("seed", [41, 42])
def test_filters_equal_oracle_on_degenerate_instances(seed):
    from paper_1211_3056_amd import _lib
    n = 4000
    A, B, N, lo, D = synth.adversarial_instances(seed, n, max_N=1 << 14)
    for alg, ref in ((_lib.HR_FILTER_LEFEVRE, lefevre_alg1), (_lib.HR_FILTER_REGULAR, regular_alg4)):
        ok, d, it = _device(alg, A, B, N, lo, D, 1)
        for i in range(n):
            bb = (int(B[i]) - int(lo[i])) % (1 << 64)
            r = ref(int(A[i]), bb, int(N[i]), int(D[i]))
            assert (int(ok[i]), int(d[i]), int(it[i])) == (int(r.success), r.d, r.iterations), (alg, i)


def test_filters_on_tabulated_exp_pieces():
    """Pieces of exp on 2^26 arguments (the Table 3 shape scaled down:
    directed, pieces of 2^15): both tests equal the oracle on every piece,
    and every piece with a degree-1 candidate is left uncertified."""
    from paper_1211_3056_amd import _lib, api, pipeline
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec("exp", 1.0, 1 << 26, 24, "dir", 1 << 15, 1 << 8, 3, 192)
    P = pipeline.UpperPrepared(spec, 4, 320)
    upper, win, thr = pipeline.upload_upper(P)
    table = pipeline.make_tables(P, upper)
    a, b = api.tabulate(table, spec.n_sub, spec.delta, spec.tau, spec.W)
    n = a.numel()
    A, B = a.cpu().numpy(), b.cpu().numpy()
    N = np.full(n, spec.N, np.uint32)
    lo = np.full(1, P.win[0], np.uint64)
    D = np.full(1, P.win[1], np.uint64)
    counts, _, _, _ = api.search(a, b, api.to_dev(N, torch.uint32), int(P.win[1]),
                                 lo=int(P.win[0]), with_inst=True)
    has_hit = counts.cpu().numpy() > 0
    assert has_hit.any()
    for alg, ref in ((_lib.HR_FILTER_LEFEVRE, lefevre_alg1), (_lib.HR_FILTER_REGULAR, regular_alg4)):
        ok, d, it = _device(alg, A, B, N, lo, D, n)
        assert not (ok.astype(bool) & has_hit).any()
        for i in range(0, n, 7):
            bb = (int(B[i]) - int(lo[0])) % (1 << 64)
            r = ref(int(A[i]), bb, spec.N, int(D[0]))
            assert (int(ok[i]), int(d[i]), int(it[i])) == (int(r.success), r.d, r.iterations), (alg, i)
