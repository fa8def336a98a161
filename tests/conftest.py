import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def otkm_gpu():
    """The HIP library binding, with a device present.  Fails (never skips) when missing."""
    from paper_2005_01182_amd import otkm
    lib = otkm.load()
    info = otkm.device_info()
    assert info["arch"].startswith("gfx950"), info
    return otkm
