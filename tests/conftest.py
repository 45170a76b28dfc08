import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(oracle.lib_path()):
        oracle.build(force=False)
    return oracle


@pytest.fixture(autouse=True, scope="module")
def _release_device_cache():
    """The full-size tests hold most of the card; return the blocks torch's
    caching allocator keeps after each module so that the next module starts
    from an empty device (nothing is initialised on a CPU-only run)."""
    yield
    if "torch" in sys.modules:
        import gc
        import torch
        if torch.cuda.is_initialized():
            gc.collect()
            torch.cuda.empty_cache()
