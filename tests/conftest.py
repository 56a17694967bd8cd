import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def load_golden(name):
    import numpy as np
    return np.loadtxt(os.path.join(ROOT, "tests", "golden", name), comments="#")


# Lines that the parity checks record (lanes compared, largest error, lanes passed by
# the conditioning guard, ties): printed in the terminal summary of every run.
PARITY_LOG = []


def pytest_terminal_summary(terminalreporter):
    if PARITY_LOG:
        terminalreporter.section("parity: lanes, largest error, conditioning guard and ties")
        for line in PARITY_LOG:
            terminalreporter.write_line(line)
