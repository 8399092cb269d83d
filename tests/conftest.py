import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def mech9_path():
    from paper_2506_02602_amd import workloads
    return workloads.mech_file("mech9")


@pytest.fixture(scope="session")
def mech32_path():
    from paper_2506_02602_amd import workloads
    return workloads.mech_file("mech32")


@pytest.fixture(scope="session")
def isomer_path():
    from paper_2506_02602_amd import workloads
    return workloads.mech_file("isomer")


@pytest.fixture(scope="session")
def omech9(mech9_path):
    import oracle
    return oracle.Mech(mech9_path)


@pytest.fixture(scope="session")
def omech32(mech32_path):
    import oracle
    return oracle.Mech(mech32_path)
