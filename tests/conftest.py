import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU checks")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.lib()  # builds the C oracle on first use if it is missing or stale
    return oracle


def _gpu_available() -> bool:
    try:
        import torch

        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def qs():
    """The HIP library binding; GPU tests only."""
    if not _gpu_available():
        pytest.skip("no GPU visible")
    import paper_2111_02396_amd as qs_mod

    qs_mod.load()  # raises if the built library is missing
    return qs_mod
