import os
import sys

import pytest

try:
    # torch's HIP runtime is mapped first, so that libcuboid (loaded by the
    # binding after torch in any case) shares it: one runtime per test process
    import torch  # noqa: F401
except ImportError:
    pass

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def golden_path(name):
    return os.path.join(GOLDEN, name)


@pytest.fixture(scope="session")
def golden():
    import json

    def load(name):
        with open(golden_path(name)) as f:
            return json.load(f)
    return load
