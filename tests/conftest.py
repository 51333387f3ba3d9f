import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def fmm():
    """The GPU library through its binding; GPU tests only."""
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2003_13218_amd as F
    F.binding.load()
    return F


def golden(name):
    """Read a golden fixture: first non-comment token of the file as float."""
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                return float(line.split()[0])
    raise ValueError(name)
