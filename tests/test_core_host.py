"""CPU checks of the device path's core arithmetic (paper_1211_3056_amd/
csrc/hr_core.h, the same __host__ __device__ code the kernels run), built
for the host with AddressSanitizer and UndefinedBehaviorSanitizer: the exact
degree-1 walk against brute force, and the device forms of the paper's
lower-bound tests (Lefevre's with swap, the unrolled regular one) against
the oracle's Alg. 1 and Alg. 4, value for value, on degenerate and random
instances."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle.search import brute_hits_np, lefevre_alg1, regular_alg4

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "core_host", "core_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("core") / "core_check")
    cmd = [hipcc, "-std=c++17", "-O1", "-g",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def _run(exe, rows):
    text = "".join(f"{a} {b} {n} {lo} {d}\n" for a, b, n, lo, d in rows)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    out = r.stdout.split("\n")
    res = []
    for i in range(len(rows)):
        h, l, g = out[3 * i].split(), out[3 * i + 1].split(), out[3 * i + 2].split()
        res.append(([int(x) for x in h[2:]], tuple(int(x) for x in l[1:]),
                    tuple(int(x) for x in g[1:])))
    return res


def _rows(seed, n, max_N):
    A, B, N, lo, D = synth.adversarial_instances(seed, n, max_N=max_N)
    return [(int(A[i]), int(B[i]), int(N[i]), int(lo[i]), int(D[i])) for i in range(n)]


@pytest.mark.parametrize("seed", [21, 22])
def test_walk_and_tests_against_oracle(checker, seed):
    rows = _rows(seed, 1500, 2500)
    # a few random slopes near the paper's workloads and large n
    g = synth.rng(seed, 3)
    for _ in range(40):
        a, b = (int(x) for x in g.integers(0, 2 ** 64, 2, dtype=np.uint64, endpoint=False))
        rows.append((a, b, int(g.integers(1 << 14, 1 << 16)), 0, 1 << 50))
    got = _run(checker, rows)
    for (a, b, n, lo, D), (hits, lef, reg) in zip(rows, got):
        assert hits == brute_hits_np(a, b, n, D, lo=lo), (a, b, n, lo, D)
        bb = (b - lo) % (1 << 64)
        ol = lefevre_alg1(a, bb, n, D)
        og = regular_alg4(a, bb, n, D)
        assert lef == (int(ol.success), ol.d, ol.iterations), (a, bb, n, D)
        assert reg == (int(og.success), og.d, og.iterations), (a, bb, n, D)
        if hits:
            assert not ol.success and not og.success       # a certified test has no hit
