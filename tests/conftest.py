import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # Run GPU tests in file order but keep the slow full-size cases late, and
    # the test_zz_* files after them (they must also pass after everything else).
    last = [i for i in items if "test_zz_" in i.nodeid]
    slow = [i for i in items if "fullsize" in i.nodeid and i not in last]
    rest = [i for i in items if i not in last and i not in slow]
    items[:] = rest + slow + last
