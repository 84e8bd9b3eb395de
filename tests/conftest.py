import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    """Build the CPU helpers (oracle, input generator) if nothing is built yet."""
    import oracle
    from paper_2002_04896_amd import synth
    if not os.path.exists(oracle.LIB):
        oracle.build()
    if not os.path.exists(synth._LIB):
        synth.build()
