import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


@pytest.fixture(autouse=True)
def _private_tune_cache(tmp_path, monkeypatch):
    """The autotuner's cache goes to a per-test file unless a test sets its own,
    so no test reads a schedule another run stored."""
    if "CHN_TUNE_CACHE" not in os.environ:
        monkeypatch.setenv("CHN_TUNE_CACHE", str(tmp_path / "chn_tune.jsonl"))
