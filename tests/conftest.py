import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU run (closed-form convergence)")


def pytest_collection_modifyitems(config, items):
    # GPU tests run in one process on a machine with the GPU; elsewhere they are skipped
    # unless explicitly selected with -m gpu (then they fail loudly).
    if os.path.exists("/dev/kfd") or "gpu" in (config.getoption("markexpr") or ""):
        return
    skip = pytest.mark.skip(reason="needs an MI355X GPU (select with -m gpu to run anyway)")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
