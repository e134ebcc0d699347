"""Shared test configuration.

Markers: ``gpu`` tests need an MI355X (gfx950) and call the HIP library through
its C-ABI; everything else runs on the CPU (oracle pins, host logic, symbol
export checks).
"""
import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

GOLDEN = ROOT / "tests" / "golden"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def golden_dir():
    return GOLDEN
