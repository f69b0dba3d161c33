import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def O():
    """The FP64 CPU oracle (built on first use)."""
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Print and flush the id of every GPU test before it touches the device,
    so a run that dies still names its case."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.stderr.write(f"\n[gpu case] {request.node.nodeid}\n")
        sys.stderr.flush()
    yield


@pytest.fixture(scope="session")
def gbk():
    """The HIP library binding; fails loudly if the library is not built or
    no GPU is present (GPU tests never fall back to anything else)."""
    import torch
    from paper_1510_01815_amd import gbk as G
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    G.load()
    return G
