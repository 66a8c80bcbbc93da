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
def rng():
    import numpy as np
    return np.random.Generator(np.random.PCG64(12345))


PACKED = os.environ.get("PCORR_TEST_PACKED_ALLOCATOR") == "1"


def pytest_collection_modifyitems(config, items):
    """GPU tests need a visible HIP device; without one they are skipped
    (the CPU suite selects -m "not gpu" anyway).  With
    PCORR_TEST_PACKED_ALLOCATOR=1 every library allocation of the session
    comes from torch's caching allocator, which packs blocks closely: a write
    past the end of a library buffer then lands in a neighbouring one and
    shows up as a parity failure instead of in allocation slack."""
    try:
        import torch
        have = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have = False
    if have:
        if PACKED:
            from paper_2304_14690_amd import pcorr
            pcorr.set_allocator(*pcorr.torch_allocator())
            for it in items:
                if "test_gpu_allocator" in it.nodeid:
                    it.add_marker(pytest.mark.skip(reason="the session installs the allocator"))
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
