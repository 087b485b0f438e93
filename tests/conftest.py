import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_sessionstart(session):
    # tests load the in-tree library: build it when none is built or when it
    # was built from other sources than the current ones
    from paper_1912_03312_amd import build as b
    if not b.is_current():
        b.build()
