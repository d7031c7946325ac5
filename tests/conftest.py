import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    return oracle.lib()


@pytest.fixture(scope="session")
def tglib():
    """The HIP library.  Built in-tree beforehand; built here only if absent."""
    from paper_2508_16522_amd import taskgraph
    if not os.path.exists(taskgraph.LIB_PATH):
        from paper_2508_16522_amd import build
        build.build_library()
    return taskgraph.load()


@pytest.fixture(scope="session")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected but no GPU is visible")
    from paper_2508_16522_amd import taskgraph
    taskgraph.load()
    return torch.device("cuda:0")
