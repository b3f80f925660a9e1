import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle case")


@pytest.fixture(scope="session", autouse=True)
def _oracle_kernel():
    """Compile the oracle's C kernel once per session if it is missing (gcc, CPU only)."""
    import oracle
    if not oracle.have_c_kernel():
        try:
            oracle.build_c_kernel()
        except Exception:  # pragma: no cover - the long-double numpy path still works
            pass
    yield
