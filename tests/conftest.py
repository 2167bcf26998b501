import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    # the parity errors the GPU tests measured, with their floors and bounds
    out = os.environ.get("ELBM_PARITY_JSON")
    if not out:
        return
    try:
        from gpu_helpers import MEASURED
    except ImportError:
        return
    import json

    with open(out, "w") as fh:
        json.dump(MEASURED, fh, indent=1)


def pytest_collection_modifyitems(config, items):
    # Run GPU tests in the order they are defined, but keep them after CPU tests
    # of the same module; nothing else to reorder.
    return
