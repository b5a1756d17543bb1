import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


@pytest.fixture(scope="session", autouse=True)
def _torch_threads():
    # the oracle's problems are small: its many small tensor ops run fastest
    # (and parallel test workers do not oversubscribe the cores) on one thread
    import torch
    torch.set_num_threads(1)


@pytest.fixture(scope="session")
def ctx():
    """A library context on cuda:0; GPU tests fail loudly without a GPU."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    import paper_2310_01775_amd as S
    c = S.Context(0)
    yield c
    c.close()
