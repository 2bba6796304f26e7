import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    # Build only when nothing is built yet; __graft_entry__.build() rebuilds on demand.
    from paper_2407_09812_amd import build as hip_build
    if not os.path.exists(hip_build.LIB):
        hip_build.build()


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle._load()
    return oracle
