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
    config.addinivalue_line("markers", "slow: full-size workloads (minutes)")


@pytest.fixture(params=["auto", "always"])
def ordered_slots(request, monkeypatch):
    """The record-slot order of single-stream decodes: the library's own rule
    (ordered slots only for streams of at least 2^22 matches), or ordered
    slots for every stream of at most 64 levels (ACEAPEX_ORDERED_SLOTS=1)."""
    if request.param == "always":
        monkeypatch.setenv("ACEAPEX_ORDERED_SLOTS", "1")
    else:
        monkeypatch.delenv("ACEAPEX_ORDERED_SLOTS", raising=False)
    return request.param
