"""GPU HR-case lists against the oracle: small ranges, config 2 in full,
config 3 and the paper's Table 3 workload against the oracle's stored full
lists.  Fused and plain forms must agree."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from conftest import golden_hr_lists
from oracle import hr as ohr
from oracle.taylor import Job

pytestmark = pytest.mark.gpu

STARTS = {"exp": 1.0, "exp2": 1.0, "log": 3.37, "sin": 1.0, "cos": 1.0}


@pytest.mark.parametrize("fname", ["exp", "exp2", "log", "sin", "cos"])
@pytest.mark.parametrize("mode", ["rn", "dir"])
def test_small_ranges_equal_bruteforce(fname, mode):
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    args = (fname, STARTS[fname], 1 << 14, 8, mode, 1 << 6, 1 << 4, 3, 128)
    ref = ohr.hr_bruteforce(Job(*args))
    assert len(ref) > 30
    fused, _ = pipeline.search_job(JobSpec(*args), "fused")
    plain, _ = pipeline.search_job(JobSpec(*args), "plain")
    assert fused == ref
    assert plain == ref


@pytest.mark.parametrize("W,delta", [(192, 3), (256, 4), (128, 2)])
def test_word_widths_and_degrees(W, delta):
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    args = ("exp", 1.125, 1 << 15, 9, "rn", 1 << 7, 1 << 5, delta, W)
    ref = ohr.hr_bruteforce(Job(*args))
    got, _ = pipeline.search_job(JobSpec(*args), "fused")
    assert got == ref


def test_config2_full_list():
    """exp on 2^32 arguments of [1, 1 + 2^-20), eps = 2^-24, RN: the GPU list
    equals the three-phase oracle's list, fused and plain."""
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec(**synth.CONFIG2)
    fused, st = pipeline.search_job(spec, "fused")
    plain, st2 = pipeline.search_job(spec, "plain")
    ref = ohr.pipeline(Job(**synth.CONFIG2))
    assert fused == ref
    assert plain == ref
    assert 400 < len(ref) < 640            # 2 eps 2^32 = 512 expected
    assert st["candidates"] == st2["candidates"]


def test_config3_full_list():
    """exp on 2^40 arguments, eps = 2^-32: the full device run; its whole HR
    list equals the oracle's stored list (tests/golden/hr_config3.txt), and
    three whole sub-intervals are recomputed by the oracle here."""
    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec(**synth.CONFIG3)
    got, st = pipeline.search_job(spec, "fused")
    assert st["pieces"] == 1 << 22
    ref = golden_hr_lists("config3")
    if ref is None:
        pytest.skip("hr_config3.txt not generated")
    assert got == ref[0]
    job = Job(**synth.CONFIG3)
    for t in (0, 1777, 4095):
        lo, hi = t * spec.per_sub, (t + 1) * spec.per_sub
        assert [m for m in got if lo <= m < hi] == ohr.pipeline(job, subs=[t])


@pytest.mark.parametrize("split", [2, 4])
def test_config3_refined_pieces_full_list(split):
    """The same 2^40 arguments with every piece split `split` ways from the
    start (pieces of N / split, the paper's phase-2 refinement applied to all
    of them), tables made on the device from the upper polynomial: fewer
    candidates, the same whole HR list as the oracle's stored one."""
    import dataclasses

    from paper_1211_3056_amd import pipeline
    from paper_1211_3056_amd.prep import JobSpec
    ref = golden_hr_lists("config3")
    if ref is None:
        pytest.skip("hr_config3.txt not generated")
    base = JobSpec(**synth.CONFIG3)
    spec = dataclasses.replace(base, N=base.N // split, tau=base.tau * split)
    got, st = pipeline.search_job(spec, "upper")
    assert st["pieces"] == (1 << 22) * split
    assert got == ref[0]


def test_paper_table3_full_list():
    """The paper's Table 3 workload: directed (53, 2^-32) HR cases of exp on
    [1, 1 + 2^-13], i.e. 2^39 + 1 binary64 arguments (its argument counts are
    twice the binary64 ones), in the batched persistent launch.  The whole
    device list equals the oracle's stored list (tests/golden/hr_table3.txt,
    241 cases; the paper prints 243)."""
    from paper_1211_3056_amd import batch
    from paper_1211_3056_amd.plan import BatchJob
    count = (1 << 39) + 1
    job = BatchJob("exp", 1.0, count, 32, "dir", sub_len=1 << 28, N=1 << 15, job_id=0)
    plan = batch.build_plan([job])
    run = batch.Runner(batch.DevicePlan(plan))
    hr = batch.finish(plan, run.batched())[0]
    assert hr == golden_hr_lists("table3")[0]
