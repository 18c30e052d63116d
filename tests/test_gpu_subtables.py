"""Sub-interval tables made on the device from a range's upper table
(hr_subtables; two levels of the hierarchical method, Sec. 5.1-5.2) against
the oracle's two-level straightforward shift, bit for bit, and the large
workload's HR list through device-made tables."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from conftest import golden_hr_lists
from oracle.tabulate import subinterval_table

pytestmark = pytest.mark.gpu


def _ints(words, W):
    L = W // 64
    return [sum(int(words[e, l]) << (64 * l) for l in range(L)) for e in range(words.shape[0])]


def _rows(flat, d):
    out, pos = [], 0
    for j in range(d + 1):
        out.append(flat[pos:pos + d - j + 1])
        pos += d - j + 1
    return out


def _device_tables(upper_words, Du, Wu, ts, Ns, delta, W, max_t=None, max_N=None):
    from paper_1211_3056_amd import api
    up = api.to_dev(upper_words.reshape(-1), torch.uint64)
    t_idx = api.to_dev(np.asarray(ts, np.uint32), torch.uint32)
    N_per = api.to_dev(np.asarray(Ns, np.uint32), torch.uint32)
    out = api.subtables(up, Du, Wu, len(ts), delta, W, N_per, t_idx=t_idx, max_t=max_t,
                        max_N=max_N)
    torch.cuda.synchronize()
    E = (delta + 1) * (delta + 2) // 2
    return out.cpu().numpy().reshape(len(ts), E, W // 64)


@pytest.mark.parametrize("Du,Wu,delta,W", [(7, 320, 4, 256), (4, 192, 3, 192), (10, 448, 6, 256),
                                          (6, 256, 2, 128), (5, 384, 5, 192), (1, 192, 1, 128)])
def test_random_upper_tables_equal_oracle(Du, Wu, delta, W):
    """Uniformly random upper words: every entry of every made table equals
    the oracle's, for uneven t and N per table (a ragged count of tables)."""
    rng = synth.rng(100 + Du * 10 + delta)
    upper = synth.random_tables(7 + Du, 1, Du, Wu)[0]
    n = 67
    max_t = min((1 << 32) - 1, int(2 ** (127.9 / Du)))
    max_N = min((1 << 32) - 1, int(2 ** ((Wu - 0.1) / Du) / delta))
    ts = rng.integers(0, max_t + 1, n).tolist()
    Ns = rng.integers(1, max_N + 1, n).tolist()
    ts[:3] = [0, 1, max_t]
    Ns[:3] = [1, max_N, 2]
    got = _device_tables(upper, Du, Wu, ts, Ns, delta, W, max_t, max_N)
    U = _rows(_ints(upper, Wu), Du)
    for r in range(n):
        ref = [v for row in subinterval_table(U, Du, ts[r], Ns[r], delta, Wu, W) for v in row]
        assert _ints(got[r], W) == ref, (r, ts[r], Ns[r])


def test_out_of_range_tables_are_zero():
    upper = synth.random_tables(3, 1, 5, 256)[0]
    got = _device_tables(upper, 5, 256, [3, 99, 4, 2], [100, 10, 1000, 0], 3, 192,
                         max_t=50, max_N=500)
    assert not got[1].any() and not got[2].any() and not got[3].any()
    assert got[0].any()


def test_product_upper_table_of_large_workload():
    """The product's upper table of exp on 2^40 arguments (degree 7, 320
    bits): device tables of sampled sub-intervals equal the oracle's shift."""
    from paper_1211_3056_amd.prep import upper_table
    c = synth.CONFIG3
    U = upper_table("exp", 1.0, c["count"], c["s"], "rn", c["N"] * c["tau"], 7, 320)
    ts = [0, 1, 2, 1777, 4094, 4095]
    got = _device_tables(U.words, 7, 320, ts, [c["N"]] * len(ts), 4, 256)
    rows = _rows(_ints(U.words, 320), 7)
    for r, t in enumerate(ts):
        ref = [v for row in subinterval_table(rows, 7, t, c["N"], 4, 320, 256) for v in row]
        assert _ints(got[r], 256) == ref, t


def test_config3_list_through_device_tables():
    """exp on 2^40 arguments, eps = 2^-32, with the 4096 sub-interval tables
    made on the device from one upper table: the whole HR list equals the
    oracle's stored list."""
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec(**synth.CONFIG3)
    got, st = pipeline.search_job(spec, "upper")
    assert st["pieces"] == 1 << 22
    ref = golden_hr_lists("config3")
    if ref is None:
        pytest.skip("hr_config3.txt not generated")
    assert got == ref[0]


def test_config2_list_through_device_tables():
    """exp on 2^32 arguments, eps = 2^-24: device-made tables give the
    oracle pipeline's list."""
    from oracle import hr as ohr
    from oracle.taylor import Job
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    got, _ = pipeline.search_job(JobSpec(**synth.CONFIG2), "upper")
    assert got == ohr.pipeline(Job(**synth.CONFIG2))
