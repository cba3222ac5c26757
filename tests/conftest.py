"""Shared test configuration.

Markers: ``gpu`` tests need an MI355X and the built HIP library; everything
else runs on the CPU.  The repository root is put on ``sys.path`` so that the
``oracle``, ``synth`` and ``paper_1108_5359_amd`` packages import without an
install step.
"""
import pathlib
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build()
    return oracle
