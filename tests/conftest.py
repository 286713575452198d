import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running (large workloads)")
    # Build the host-only helper libraries if they are missing (seconds, gcc).
    from synth import build as sb
    from oracle import build as ob
    if not os.path.exists(os.path.join(ROOT, "synth", "libsynth.so")):
        sb.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        ob.build()


@pytest.fixture
def rng():
    import numpy as np
    return np.random.default_rng(12345)
