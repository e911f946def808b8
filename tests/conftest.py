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
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def pytest_runtest_logstart(nodeid, location):
    # Name the case before it touches the GPU, so a fault still leaves its name behind.
    if os.environ.get("EVQ_ANNOUNCE"):
        print(f"\n[start] {nodeid}", flush=True)


@pytest.fixture
def tuned():
    """Setter of the library's scheduling knobs (evq_tuning) for one test; restored after it."""
    import paper_2502_10579_amd as evq
    prev = evq.get_tuning()
    yield evq.set_tuning
    evq.set_tuning(**prev)
