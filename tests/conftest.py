import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


_torch_cuda_ready = False


@pytest.fixture(autouse=True)
def _torch_cuda_first(request):
    """Before the first GPU test of a session, let torch initialise its own
    HIP runtime (torch ships one beside the system runtime the library
    uses): on this image a torch initialisation that comes after the library
    and the oracle have run in the process can report no GPU."""
    global _torch_cuda_ready
    if not _torch_cuda_ready and request.node.get_closest_marker("gpu") is not None:
        import torch
        torch.cuda.init()
        _torch_cuda_ready = True
    yield

