import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: larger host-side cases")


def load_golden_matrices(name):
    """Parse a tests/golden/*.txt fixture of [NAME] blocks of integer rows."""
    import numpy as np
    blocks, cur = {}, None
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                cur = line.strip("[]")
                blocks[cur] = []
            else:
                blocks[cur].append([int(x) for x in line.split()])
    return {k: np.array(v, dtype=np.int64) for k, v in blocks.items()}
