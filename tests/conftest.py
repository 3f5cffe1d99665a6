import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session", autouse=True)
def _librfps_built():
    """Builds librfps.so once if it is missing (a fresh checkout); an existing
    build is used as it is."""
    from paper_2606_06255_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()
