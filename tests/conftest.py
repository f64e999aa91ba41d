import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: longer CPU test")


TUNE_KEYS = ("LE_TUNE_ROW", "LE_TUNE_ROW_FWD", "LE_TUNE_ADV", "LE_TUNE_MU", "LE_TUNE_COL_CH",
             "LE_TUNE_COL_FLOW")


@pytest.fixture
def fixed_variants(monkeypatch):
    """Fix every autotuned kernel variant (to the fused / default shapes) for
    tests that compare two contexts bit for bit: equal results need equal
    variants, and the autotuner times each context on its own."""
    for k in TUNE_KEYS:
        monkeypatch.setenv(k, "0")
    return monkeypatch
