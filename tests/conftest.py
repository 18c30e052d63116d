import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def read_golden(name):
    """Non-comment lines of a golden fixture, split at '|' when present."""
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            out.append(line)
    return out


@pytest.fixture
def golden():
    return read_golden


def golden_hr_lists(name):
    """HR-case lists of tests/golden/hr_<name>.txt (written by
    tests/golden/make_lists.py from the oracle alone): {job id: sorted
    offsets m}, or None when the file has not been generated."""
    path = os.path.join(GOLDEN, f"hr_{name}.txt")
    if not os.path.exists(path):
        return None
    out = {}
    for line in read_golden(f"hr_{name}.txt"):
        head, tail = line.split("|")
        jid = int(head.split()[0])
        lst = out.setdefault(jid, [])
        m = tail.split()[0]
        if m != "-":
            lst.append(int(m))
    return {j: sorted(v) for j, v in out.items()}
