import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
    # The CPU-side libraries are cheap to build; build them only when missing.
    # The GPU library is never built here: build() does that before a run.
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        from oracle import build as ob
        ob.build()
    if not os.path.exists(os.path.join(ROOT, "paper_1204_6255_amd", "graphgen", "libdigen.so")):
        from paper_1204_6255_amd.graphgen import build as gb
        gb.build()
