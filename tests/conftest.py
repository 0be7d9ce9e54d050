import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """Library context on cuda:0 for the whole GPU session (nonblocking;
    tests switch modes with GrM_set_mode and restore it)."""
    import torch
    from paper_2509_14211_amd import api, grb
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    grb.load()
    ctx = api.Context(grb.GrB_NONBLOCKING)
    ctx.__enter__()
    yield grb
    ctx.__exit__(None, None, None)


@pytest.fixture()
def nonblocking(gpu):
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
    yield gpu
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)


@pytest.fixture()
def blocking(gpu):
    gpu.GrM_set_mode(gpu.GrB_BLOCKING)
    yield gpu
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
