"""CPU checks of bench.py's command line (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def test_ops_model_counts_each_phase():
    """The algorithmic-ops model adds the tabulation, walk and recheck terms:
    each term is zero when its count is, and a 256-bit table pays the top-128
    rejection for every candidate and the full width only where asked."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1211_3056_amd.prep import JobSpec
    spec = JobSpec("exp", 1.0, 1 << 20, 32, "rn", 1 << 10, 1 << 4, 4, 256)
    tab = bench.ops_model(spec, 1, 0, 0, 0)
    assert tab == (4 + 3 + 2 + 1 + 0) * 8            # sum_j (delta - j) limb adds, L = 8
    assert bench.ops_model(spec, 0, 0, 1, 0) == 96
    top = bench.ops_model(spec, 0, 1, 0, 0)
    full = bench.ops_model(spec, 0, 0, 0, 1)
    assert top == 4 * (2 * (4 + 3 + 2 + 1) + 4) + 12
    assert full == 4 * (2 * (8 + 7 + 6 + 5) + 8) + 12
    assert bench.ops_model(spec, 2, 3, 5, 7) == 2 * tab + 3 * top + 5 * 96 + 7 * full
