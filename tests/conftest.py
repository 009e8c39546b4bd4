import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def cfg_small():
    from wvgen import get_config
    return get_config("gray64")


@pytest.fixture(scope="session")
def weights_small(cfg_small):
    from wvgen import make_weights
    return make_weights(cfg_small)


@pytest.fixture(scope="session")
def cfg_big():
    from wvgen import get_config
    return get_config("ycbcr512x768")


@pytest.fixture(scope="session")
def weights_big(cfg_big):
    from wvgen import make_weights
    return make_weights(cfg_big)
