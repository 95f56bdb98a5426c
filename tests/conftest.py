import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def read_golden(name):
    """key = value lines of tests/golden/<name>, comments after '#' dropped."""
    vals = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            vals[k] = v
    return vals


@pytest.fixture(scope="session")
def golden_paper():
    return read_golden("paper_values.txt")


@pytest.fixture(scope="session")
def native():
    """The built library (built here only if nothing is built yet)."""
    from paper_1201_5380_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_1201_5380_amd import build
        build.build()
    return _native.lib()


@pytest.fixture(scope="session")
def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")
