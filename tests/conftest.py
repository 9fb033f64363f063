import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _gpu_available() -> bool:
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library shares)
        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu_lib():
    """The C-ABI library on a real GPU; GPU tests fail loudly without it."""
    if not _gpu_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    from paper_2303_03681_amd import binding
    return binding.load()
