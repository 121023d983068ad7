import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X (gfx950)")
    config.addinivalue_line("markers", "slow: long-running test")
    # The plain-C helpers are cheap to compile; build them only when absent.
    import oracle
    import synth
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build_lib()
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        synth.build_lib()
