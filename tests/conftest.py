import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~10 s")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    """The HIP library binding; GPU tests fail loudly if it is not built."""
    import paper_2206_00975_amd as nsk
    nsk.load()
    return nsk


# GPU tests of the batched persistent kernel (see their skip marks)
BATCHED_FAULT = ("the batched kernel once ended in an illegal-address GPU fault in a batch of FP64 "
                 "instances after passing every earlier run; the cause is not established, so its "
                 "tests stay skipped until it is")
