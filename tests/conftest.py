import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))
for _p in (ROOT, TESTS):          # the package, the oracle, and test helpers shared between files
    if _p not in sys.path:
        sys.path.insert(0, _p)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle as O
    O._load()
    return O


@pytest.fixture(autouse=True, scope="session")
def _hip_runtime_before_oracle():
    """Initialise the library's HIP runtime before any test runs the oracle
    with many OpenMP threads: on the MI355X machine a first HIP initialisation
    after a 16-thread OpenMP region reported no device."""
    try:
        import torch
        if torch.cuda.is_available():
            from paper_1012_2865_amd import moray as M
            M.moray_free(M.moray_init(device=0))
    except Exception:
        pass
    yield
