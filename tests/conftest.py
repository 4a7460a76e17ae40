import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def cfg1_problem():
    from pdg_inputs import problems
    return problems.cfg1()


@pytest.fixture(scope="session")
def cfg1_oracle(cfg1_problem):
    from oracle.monodomain import Monodomain
    return Monodomain(cfg1_problem)


@pytest.fixture(scope="session")
def small3d_problem():
    from pdg_inputs import problems
    return problems.small3d()


@pytest.fixture(scope="session")
def small3d_oracle(small3d_problem):
    from oracle.monodomain import Monodomain
    return Monodomain(small3d_problem)
