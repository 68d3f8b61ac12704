import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def mech_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("mech")


@pytest.fixture(scope="session")
def c0_path(mech_dir):
    return synth.write_mechanism(synth.MECH_C0, str(mech_dir / "c0.mech"))


@pytest.fixture(scope="session")
def c1_path(mech_dir):
    return synth.write_mechanism(synth.MECH_C1, str(mech_dir / "c1.mech"))
