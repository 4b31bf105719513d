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


def say(config, msg):
    """Write a line to the terminal past pytest's output capture (progress of
    long GPU cases, and the case that was running if a run ends abruptly)."""
    capman = config.pluginmanager.getplugin("capturemanager")
    if capman is None:
        sys.stderr.write(msg + "\n")
        sys.stderr.flush()
        return
    with capman.global_and_fixture_disabled():
        sys.stderr.write(msg + "\n")
        sys.stderr.flush()


@pytest.fixture(autouse=True)
def _announce_gpu_case(request):
    """Name each GPU case on the terminal before it runs."""
    if request.node.get_closest_marker("gpu") is not None:
        say(request.config, f"\n[gpu-case] {request.node.nodeid}")
    yield


@pytest.fixture
def progress(request):
    """progress(msg): a line on the terminal during a long test."""
    return lambda msg: say(request.config, msg)


@pytest.fixture(scope="session")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_1010_3816_amd import binding

    return binding
