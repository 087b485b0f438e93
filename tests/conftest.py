import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_sessionstart(session):
    # tests load the in-tree library; build it only when nothing is built
    lib = os.path.join(ROOT, "paper_1912_03312_amd", "librexi.so")
    if not os.path.exists(lib):
        from paper_1912_03312_amd.build import build
        build()
