import os
import sys

import pytest

try:  # imported at collection so a slow first import is not charged to a test
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU-only checks")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """The HIP library on cuda:0. Skips when no GPU is visible; raises when the
    GPU is there but the library is not built (no silent fallback)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_1603_02421_amd as sph
    sph.native.load()  # raises if libsphjet.so is missing
    return sph
