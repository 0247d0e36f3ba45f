import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line(
        "markers", "slow: takes more than a few seconds on the CPU")


def load_golden(name):
    """Parse tests/golden/<name>: rows 'label | n | input | output'."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            label, n, xin, yout = (p.strip() for p in line.split("|"))

            def parse(s):
                vals = []
                for tok in s.split():
                    re, im = tok.split(",")
                    vals.append(complex(float(re), float(im)))
                return np.array(vals, dtype=np.complex128)
            rows[label] = (int(n), parse(xin), parse(yout))
    return rows
