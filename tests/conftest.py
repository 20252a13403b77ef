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
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    # the generator and the oracle are plain C; build them if nothing is built yet
    import dcgen
    import oracle
    if not os.path.exists(dcgen.LIB_PATH):
        dcgen.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
