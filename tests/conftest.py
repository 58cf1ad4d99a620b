import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle runs")


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available() and torch.cuda.device_count() > 0
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _have_gpu():
        return
    skip = pytest.mark.skip(reason="no GPU device in this process")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def load_golden_matrices(path):
    import numpy as np
    mats = {}
    with open(path) as f:
        lines = [l.strip() for l in f if l.strip() and not l.startswith("#")]
    i = 0
    while i < len(lines):
        name, dim = lines[i].split()
        dim = int(dim)
        rows = [[complex(v) for v in lines[i + 1 + r].split()] for r in range(dim)]
        mats[name] = np.array(rows, dtype=complex)
        i += 1 + dim
    return mats
