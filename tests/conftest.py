import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import ref
    ref.build()
    return ref


@pytest.fixture(autouse=True)
def _no_tune_cache_file(monkeypatch):
    """Tests tune afresh: no tuning cache file is read or written unless a test
    names one itself."""
    if "BDIS_TUNE_CACHE" not in os.environ:
        monkeypatch.setenv("BDIS_TUNE_CACHE", "")
