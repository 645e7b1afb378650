import os
import sys

import pytest

# Load torch's HIP runtime before the library (the benchmark does the same):
# both provide libamdhip64.so.7, and the process must use one of them for the
# library and for torch (the autograd wrapper) alike.
try:
    import torch  # noqa: F401
except ImportError:
    pass

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def smrt_mod():
    from paper_2504_21784_amd import smrt
    smrt.load()
    return smrt
