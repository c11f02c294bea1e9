import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _native_helpers():
    """Build the CPU-side helpers (reference decoder, workload encoder) if absent."""
    import oracle
    from paper_cs_0605069_amd import workloads

    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    if not os.path.exists(os.path.join(ROOT, "paper_cs_0605069_amd", "workloads", "libgfsynth.so")):
        workloads.build_native()
    yield
