import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# GPU tests run the VM in checked mode: every map-value access is compared
# against the bounds of the map it was verified against.
os.environ.setdefault("GX_CHECKED", "1")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) GPU")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    yield
