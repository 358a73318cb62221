import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def tmpdir_session(tmp_path_factory):
    return tmp_path_factory.mktemp("nep")


def write_model(tmpdir, name, model):
    from paper_2409_04430_amd import inputs as I
    path = os.path.join(str(tmpdir), name + ".nep")
    I.write_model(path, model)
    return path


def cluster_box():
    return np.array([60.0, 60.0, 60.0])
