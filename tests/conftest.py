import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    return oracle


def pytest_terminal_summary(terminalreporter):
    from tests.metrics import REPORT
    if REPORT:
        terminalreporter.section("errors against the FP64 oracle (peak-normalised |f|^2, per transition)")
        for line in REPORT:
            terminalreporter.write_line(line)
