import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-only check, skipped unless FSIM_SLOW=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("FSIM_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow; set FSIM_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
