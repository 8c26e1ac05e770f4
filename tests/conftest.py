import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (large workloads)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    if not os.path.exists(os.path.join(ROOT, "oracle", "libaptoracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def synth():
    import aptsynth

    if not os.path.exists(os.path.join(ROOT, "aptsynth", "libaptsynth.so")):
        aptsynth.build()
    return aptsynth
