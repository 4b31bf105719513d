"""Test configuration: the `gpu` marker and one-time build of missing libraries."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _ensure_built():
    # Build only what is missing; a present library is used as it is.
    import __graft_entry__ as ge

    if not os.path.exists(ge.ORACLE_LIB):
        ge.build_oracle()


_ensure_built()


@pytest.fixture(scope="session")
def orc():
    import oracle

    return oracle


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name each GPU case on the real stderr before it runs, so that a run
    that ends abruptly still says which case was executing."""
    if request.node.get_closest_marker("gpu") is not None:
        sys.__stderr__.write(f"\n[gpu-case] {request.node.nodeid}\n")
        sys.__stderr__.flush()
    yield


@pytest.fixture(scope="session")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_1010_3816_amd import binding

    return binding
