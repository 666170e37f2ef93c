import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """Parse a golden fixture: '#' comments, then whitespace-separated key value pairs."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


@pytest.fixture
def golden():
    return read_golden


def decision_cases(read):
    """The hand-derived decision cases: name -> (A, expected, options), where expected
    is (s, k, n_est) or an error code such as "ENOCONV" and options holds max_sqrt and
    k_max (5 unless the line sets it: most cases were derived for schemes 1..5)."""
    import numpy as np

    out = {}
    for name, (mat, n, s, k, nest, *opts) in read("decisions.txt").items():
        kw = dict(o.split("=", 1) for o in opts)
        A = np.array([float(v) for v in mat.split(",")]).reshape(int(n), int(n))
        expected = kw["status"] if "status" in kw else (int(s), int(k), int(nest))
        out[name] = (A, expected, {"max_sqrt": int(kw.get("max_sqrt", 50)),
                                   "k_max": int(kw.get("k_max", 5))})
    return out
