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
def oracle_mod():
    import oracle
    oracle._load()
    return oracle


@pytest.fixture(scope="session")
def gen():
    from paper_2408_05238_amd import inputs
    inputs._load()
    return inputs


try:  # import torch during collection so the first GPU test's timeout excludes it
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
