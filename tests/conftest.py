import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def gpu_lib():
    """The product library, loaded for GPU tests; fails loudly if missing."""
    from paper_2010_08695_amd import tip
    lib = tip.load()
    if not tip.device_available():
        pytest.fail("no HIP device visible to libtip")
    return lib
