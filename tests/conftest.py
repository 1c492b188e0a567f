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
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "fullsize: full-size parity against the oracle (minutes of host time)")


@pytest.fixture(scope="session")
def blosum():
    from workloads import blosum62
    return blosum62()


@pytest.fixture(scope="session")
def dna():
    from workloads import dna_matrix
    return dna_matrix(2, -3)
