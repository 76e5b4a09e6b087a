import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device); parity and device tests")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0; tests marked gpu skip only where no GPU
    exists at all (the CPU suite deselects them anyway)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this host")
    from paper_1806_10241_amd import axlb
    axlb.load()
    return torch


def say(*a):
    """Progress line that names the GPU case about to run."""
    print(*a, flush=True)


def golden(name):
    """Rows of a fixture under tests/golden/ (values the paper prints; the
    file header cites the table): list of tuples of str."""
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append(tuple(line.split()))
    return rows
