import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test taking more than ~20 s")


@pytest.fixture(scope="session")
def k10():
    from oracle.constants import wavenumber
    return wavenumber(10.0e9)


@pytest.fixture(scope="session")
def unit1():
    from workloads.mesh import macro_unit
    return macro_unit((0.006, 0.009))


@pytest.fixture(scope="session")
def unit2():
    from workloads.mesh import macro_unit
    return macro_unit((0.005, 0.007, 0.009, 0.011))
