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
def _one_hip_runtime():
    """Load torch's HIP runtime, then create and free one library context, at
    the start of a GPU session: the library then runs on torch's runtime (the
    binding imports torch before it loads the library; a second HIP runtime
    loaded into the same process leaves the one initialised last without a
    device)."""
    try:
        import torch
        if torch.cuda.is_available():
            from paper_1012_2865_amd import moray as M
            M.moray_free(M.moray_init(device=0))
    except Exception:
        pass
    yield
