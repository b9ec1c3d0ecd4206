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
    """The CPU helper libraries (input generator, oracle) are built on demand."""
    import oracle
    import synth
    for mod in (synth, oracle):
        if not os.path.exists(mod._LIB):
            mod.build()
    yield
