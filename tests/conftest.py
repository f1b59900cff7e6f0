import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # Run GPU tests in file order but keep the slow full-size cases last.
    slow = [i for i in items if "fullsize" in i.nodeid]
    rest = [i for i in items if "fullsize" not in i.nodeid]
    items[:] = rest + slow
