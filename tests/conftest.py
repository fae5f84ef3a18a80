import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU runs")


@pytest.fixture(scope="session")
def oracle():
    from oracle import adref
    if not adref.LIB.exists():
        adref.build()
    return adref


@pytest.fixture(scope="session")
def golden_dir():
    return ROOT / "tests" / "golden"
