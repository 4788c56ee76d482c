import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle (built on first use only when no library is present)."""
    from oracle import oracle as o
    if not o.LIB_PATH.exists():
        o.build()
    return o


@pytest.fixture(scope="session")
def inputs():
    from paper_0805_1827_amd import inputs as m
    return m


def cpu_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 16))
