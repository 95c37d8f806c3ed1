import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session", autouse=True)
def _built_helpers():
    """The CPU helpers (input generator, oracle) are tiny gcc builds; build
    them if a fresh checkout has no binaries yet."""
    import datagen
    import oracle
    datagen.build(force=False)
    oracle.build(force=False)
    yield
