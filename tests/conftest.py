import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    # the library is built in-tree; build it only when nothing is there
    lib = os.path.join(ROOT, "paper_1506_05996_amd", "libsem.so")
    if not os.path.exists(lib):
        from paper_1506_05996_amd.build import build
        build(verbose=False)
